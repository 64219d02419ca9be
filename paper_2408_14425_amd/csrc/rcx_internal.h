// rcx_internal.h -- shared declarations of librcx's host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/rcx.h"

namespace rcx {

// Unsigned division by a launch constant d >= 1: q = n / d for every 32-bit
// n with one high multiply, two shifts and two adds (Granlund and
// Montgomery 1994, the round-up method; the 33-bit multiplier is 2^32 + m).
struct FastDiv {
    uint32_t d = 1, m = 1, s1 = 0, s2 = 0;
    __host__ __device__ uint32_t div(uint32_t n) const
    {
        const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
        return (t + ((n - t) >> s1)) >> s2;
    }
};

inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d < 1 ? 1 : d;
    uint32_t l = 0;
    while ((1ull << l) < f.d) ++l;  // ceil(log2 d)
    f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - f.d)) / f.d + 1);
    f.s1 = l > 0 ? 1 : 0;
    f.s2 = l > 0 ? l - 1 : 0;
    return f;
}

constexpr uint32_t kDecodeReady = 0x52435844u;

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
    // Launch order of the rays: 0 = probe-major (direction fastest); else
    // groups of tile_p x tile_p probes x tile_d directions, so the rays a
    // launch runs at one time cross a compact band of cells.
    int32_t tile_p, tile_d;
    // 1: the field march of a tiled order with an even tile_p runs the 4
    // rows of a wavefront on one direction and shares their cell walk
    // (march_rows.h, k_march_shared; bitwise the same results), else one
    // walk per row
    int32_t shared_walk = 0;
    // workgroups are given to the 8 XCDs in chunks of xcd_chunk consecutive
    // ones (march_rows.h, xcd_block_chunked)
    int32_t xcd_chunk = 128;
    // path length per unit of projected (x-z) length: 1 / sin(theta) for a
    // ray inclined at theta to the invariant y axis; 1 in flatland
    double ds_scale = 1.0;
    // sparse solve: the flagged probes (v * px + u) whose rays are marched,
    // n_active of them, in the launch order's probe order (tile by tile when
    // tile_p > 0); nullptr = every probe
    const int32_t* plist = nullptr;
    int32_t n_active = 0;
    // Divisors of the ray-index decode (march_rows.h, ray_coords) and of the
    // XCD order, set by set_decode() on the host before every launch.
    struct Decode {
        FastDiv nd, px, per, nw, tile_d, tile_p, ntx, tp2, chunk, chunk8;
        uint32_t ready = 0;
    } dec;
};

// Rays a march launch covers (the tiled order pads the probe grid to whole
// tiles; padding rays are inactive).
inline int64_t level_launch_rays(const LevelDesc& L)
{
    if (L.plist) {
        const int64_t per = L.tile_p > 0 ? (int64_t)L.tile_p * L.tile_p : 1;
        return (L.n_active + per - 1) / per * per * L.nd;
    }
    if (L.tile_p <= 0) return (int64_t)L.px * L.pz * L.nd;
    const int64_t tx = (L.px + L.tile_p - 1) / L.tile_p, tz = (L.pz + L.tile_p - 1) / L.tile_p;
    return tx * tz * L.tile_p * L.tile_p * L.nd;
}

// Fill L.dec from the launch order and the XCD chunk. False (and L.dec not
// ready) when the launch's ray indices would not fit in 31 bits.
inline bool set_decode(LevelDesc& L)
{
    LevelDesc::Decode& D = L.dec;
    D.ready = 0;
    if (level_launch_rays(L) >= ((int64_t)1 << 31) || L.nd < 1 || L.px < 1 || L.xcd_chunk < 1) return false;
    D.nd = make_fastdiv((uint32_t)L.nd);
    D.px = make_fastdiv((uint32_t)L.px);
    if (L.tile_p > 0) {
        D.per = make_fastdiv((uint32_t)(L.tile_p * L.tile_p * L.tile_d));
        D.nw = make_fastdiv((uint32_t)(L.nd / L.tile_d));
        D.tile_d = make_fastdiv((uint32_t)L.tile_d);
        D.tile_p = make_fastdiv((uint32_t)L.tile_p);
        D.ntx = make_fastdiv((uint32_t)((L.px + L.tile_p - 1) / L.tile_p));
        D.tp2 = make_fastdiv((uint32_t)(L.tile_p * L.tile_p));
    }
    D.chunk = make_fastdiv((uint32_t)L.xcd_chunk);
    D.chunk8 = make_fastdiv((uint32_t)L.xcd_chunk * 8u);
    D.ready = kDecodeReady;
    return true;
}

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
// smax_bits (nullable): [n_batch * batch_width] per-wavelength max of S (float bits).
hipError_t launch_prep(const float* chi, const float* eta, float2* F, int32_t n_wave, int64_t ncell,
                       float voxel, unsigned int* smax_bits, hipStream_t st);
// Input checks (RCX_FLAG_CHECK_INPUT): zero *flag, then OR into it 1 for a
// non-finite value and 2 for a finite one out of the range among a[0..n).
constexpr int32_t kCheckNonNegative = 0;  // v >= 0
constexpr int32_t kCheckPositive = 1;     // v > 0
constexpr int32_t kCheckFinite = 2;       // any finite v
hipError_t launch_zero_flag(unsigned int* flag, hipStream_t st);
// p[0..n) = v.
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_check_f32(const float* a, int64_t n, int32_t range, unsigned int* flag, hipStream_t st);
hipError_t launch_check_f64(const double* a, int64_t n, int32_t range, unsigned int* flag, hipStream_t st);
// Read the flag back (synchronises st): RCX_OK if 0, else RCX_E_NONFINITE
// with a message naming `what`.
int32_t check_flag_result(const unsigned int* flag, const char* what, hipStream_t st);
// Exponent biases of the 16-bit cascade storage from the per-wavelength
// max S: ebias = E(max S) - 62, E the FP32 exponent field.
hipError_t launch_ebias(int32_t n, const unsigned int* smax_bits, int32_t* ebias, hipStream_t st);

// Cascade buffers of one march launch: the merged cascade above (read) and
// this cascade (written), each FP32 or 16-bit codes with exponent biases.
struct CascIO {
    const void* up;
    void* out;
    bool up_f16, out_f16;
    const int32_t* ebias_b;    // [batch_width] exponent biases of the 16-bit codes (2 x with pairs)
    int64_t slot_stride = 0;   // pairs of batches: elements from batch b's cascade to b+1's
};
// Wavelengths per batch of the field and cascade layouts.
int32_t batch_width();
// Grid of a march launch over `rays` rays.
dim3 march_grid(int64_t rays);
// Fb: the batch's slice of F ([ncell][batch_width] float2); up/out: cascade
// buffers [rays][batch_width]. With io.slot_stride != 0 the launch marches
// batches b and b+1 together (the next slice of F; cascades slot_stride
// elements further on).
hipError_t launch_march_merge(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                              const CascIO& io, hipStream_t st);
// Cascade 0 with 4 directions: march, merge and J in one launch (no stored
// cascade 0): J[lam0 + l][c] for l < n_valid, and with a pair also
// J[lam0 + batch_width + l][c] for l < n_valid1.
hipError_t launch_march_merge_j(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                const CascIO& io, float* J, int32_t lam0, int32_t n_valid, int32_t n_valid1,
                                float w, bool acc, hipStream_t st);
// Bilinear fix (io.slot_stride != 0: batches b and b+1 per lane, as in
// launch_march_merge): interval (p, k) traced
// once per bilinear probe q of the cascade above, to q + t_b w_k, merged
// with q's children and summed with the bilinear weights; up/out as for
// launch_march_merge. Needs a cascade above in the plan (qx, qz, nd_up).
hipError_t launch_march_fix(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                            const CascIO& io, hipStream_t st);
// kInclSlots inclinations per lane in one launch (FP32 cascades, slot w
// io.slot_stride * w elements on): sc[w] = path per projected cell, wt[w]
// the quadrature weights (cascade 0 with 4 directions writes J).
constexpr int kInclSlots = 8;
hipError_t launch_march_merge_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                   const CascIO& io, const float* sc, hipStream_t st);
// The bilinear fix with the kInclSlots inclinations as slots (FP32).
hipError_t launch_march_fix_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                 const CascIO& io, const float* sc, hipStream_t st);
hipError_t launch_march_merge_j_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb,
                                     const double4* dirs, const CascIO& io, float* J, int32_t lam0, int32_t n_valid,
                                     const float* sc, const float* wt, hipStream_t st);
// Sparse solve: zero the field batches F [n_batch][ncell][16] at cells
// with mask 0 (transparent, no emission), and J [n_wave][ncell] there.
hipError_t launch_mask_fields(float2* F, const uint8_t* mask, int64_t ncell, int32_t n_batch, hipStream_t st);
hipError_t launch_mask_j(float* J, const uint8_t* mask, int64_t ncell, int32_t n_wave, hipStream_t st);
// J[lam0 + l][c] = (1/n0) sum_k I0[(c * n0 + k)][l] for l < n_valid.
// The J writers take a weight w and acc: J = w * value, or J += w * value
// (inclination quadrature: one pass per inclination).
hipError_t launch_j(const float* I0, float* J, int32_t lam0, int32_t n_valid, int64_t ncell, int32_t n0, float w,
                    bool acc, hipStream_t st);

}  // namespace rcx

#include <vector>

// A formal-solve plan: grid, cascade geometry and the device direction table.
struct rcx_plan {
    rcx_grid grid;
    rcx_params prm;
    int32_t max_wave;
    int32_t n_casc;
    int32_t top_skipped;
    std::vector<rcx::LevelDesc> levels;
    // inclination quadrature (Gauss-Radau in mu = cos(angle to y) on [0, 1],
    // fixed node mu = 0): path scale 1/sqrt(1 - mu^2) and weight per node
    std::vector<double> incl_scale, incl_w;
    std::vector<int32_t> dir_off;  // offset of cascade i's directions in the table
    std::vector<double4> dirs_host;
    double4* dirs_dev = nullptr;
    // sparse solve (rcx_plan_set_active_host): cascade-0 mask and the
    // flagged probe lists of every cascade (levels[i].plist points here)
    uint8_t* mask_dev = nullptr;
    int32_t* plist_dev = nullptr;
    std::vector<uint8_t> active_host;  // the flags last given (the lists follow the launch order)
    void* ws_own = nullptr;
    size_t ws_own_bytes = 0;
    void* scratch = nullptr;  // the library's scratch on the plan's device (rcx_formal_solve_noalloc)
    bool work_done = false;
    rcx_work work;
    // measurement: events recorded around launches when timing is enabled
    struct Timed {
        int32_t level;  // cascade index, or -1 for prep / J
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<Timed> pending;
    int64_t n_solves = 0;
    int64_t n_march_enqueued = 0;  // march launches enqueued since plan_enqueue_solve began
};

namespace rcx {
// The formal solve of rcx_formal_solve on the plan's own workspace, enqueue
// only: no argument or input check and no synchronisation, so a stream
// capture may record it (the batched path runs its large atmospheres
// through it). *march_launches (nullable) receives the march launches it
// enqueued.
int32_t plan_enqueue_solve(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, float* J,
                           hipStream_t st, int64_t* march_launches);
}  // namespace rcx


