// rcx_plan.hip -- host side of librcx: plans, cascade geometry, work counts
// and the orchestration of one formal solve (Osborne & Sannikov,
// arXiv:2408.14425, Secs. 2.3-2.4 and 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "incl_quadrature.h"
#include "rcx_internal.h"

namespace rcx {

// Ray order of the upper cascades (see LevelDesc::tile_p).
constexpr int32_t kTileMinDirs = 256;
// Cascades marched two wavelength batches at a time (see rcx_formal_solve).
constexpr int32_t kPairMaxDirs = 256;
constexpr int32_t kTileProbes = 4;
constexpr int32_t kTileDirs = 32;

// The allocation-free formal solve's scratch (rcx_formal_solve_noalloc):
// a file-scope device array, one copy per GPU, held until the process ends.
// Host code uses only the device address that hipGetSymbolAddress returns
// for the current device (kept per device in g_scratch), never the array's
// name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
thread_local int32_t g_last_code = RCX_OK;
thread_local char g_last_msg[512] = "";
}  // namespace

int32_t fail(int32_t code, const std::string& msg)
{
    g_last_code = code;
    std::snprintf(g_last_msg, sizeof(g_last_msg), "%s", msg.c_str());
    return code;
}

int32_t hip_fail(hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return fail(RCX_E_HIP, m);
}

static int32_t ok()
{
    g_last_code = RCX_OK;
    g_last_msg[0] = 0;
    return RCX_OK;
}

// Device address of the scratch array on the current device, looked up
// once per device (at plan creation: rcx_plan_create calls this with the
// plan's device current).
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

int32_t scratch_address(void** out)
{
    *out = nullptr;
    int dev = 0;
    RCX_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RCX_E_UNSUPPORTED, "scratch: device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return RCX_OK;
}

int32_t check_flag_result(const unsigned int* flag, const char* what, hipStream_t st)
{
    unsigned int h = 0u;
    RCX_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
    RCX_HIP_TRY(hipStreamSynchronize(st));
    if (h == 0u) return RCX_OK;
    std::string m = std::string(what) + ":";
    if (h & 1u) m += " a value is not finite";
    if (h & 2u) m += (h & 1u) ? "; a value is out of range" : " a value is out of range";
    return fail(RCX_E_NONFINITE, m);
}

}  // namespace rcx

using namespace rcx;

namespace {

double t_start(const rcx_params& p, int32_t n_casc, int32_t i)
{
    if (i <= 0) return 0.0;
    if (i >= n_casc) return INFINITY;
    if (p.t_rule == RCX_T_LENGTH_X4) return p.c0_t1 * (std::ldexp(1.0, 2 * i) - 1.0) / 3.0;
    return p.c0_t1 * std::ldexp(1.0, 2 * (i - 1));
}

int32_t auto_cascades(int32_t nx, int32_t nz)
{
    int32_t m = std::max(nx, nz), k = 0;
    while ((int64_t(1) << (2 * k)) < m) ++k;
    return k + 2;
}

int64_t level_entries(const LevelDesc& L) { return (int64_t)L.px * L.pz * L.nd; }

// Largest distance from any probe of a cascade to any corner of the domain:
// a cascade whose interval starts beyond it has only empty rays.
double max_probe_corner_distance(const rcx_grid& g, const LevelDesc& L)
{
    double best = 0.0;
    const double us[2] = {0.5 * L.s, (L.px - 0.5) * L.s};
    const double vs[2] = {0.5 * L.s, (L.pz - 0.5) * L.s};
    const double xs[2] = {0.0, (double)g.nx};
    const double zs[2] = {0.0, (double)g.nz};
    for (double u : us)
        for (double v : vs)
            for (double x : xs)
                for (double z : zs) best = std::max(best, std::hypot(u - x, v - z));
    return best;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct WsLayout {
    size_t F, casc_a, casc_b, smax, ebias, flag, total;
    int64_t casc_slot;  // elements of one batch's slot in a cascade buffer
};

// The paper's 8 inclinations with FP32 cascades run as slots of one march
// (one walk and one field load per step for all 8); other counts, or FP16
// cascades, run one pass per inclination.
bool incl_slots(const rcx_plan* p) { return p->prm.n_incl == kInclSlots && p->prm.storage == RCX_STORE_F32; }

WsLayout ws_layout(const rcx_plan* p, int32_t n_wave)
{
    WsLayout w{};
    const int64_t ncell = (int64_t)p->grid.nx * p->grid.nz;
    int64_t max_entries = 0;
    for (const auto& L : p->levels) max_entries = std::max(max_entries, level_entries(L));
    const int64_t lb = batch_width();
    const int64_t n_batch = (n_wave + lb - 1) / lb;
    // two batches are marched together when there are at least two: each
    // cascade buffer then holds both (slot 1 at casc_slot elements)
    const int64_t slots = incl_slots(p) ? kInclSlots : (n_batch >= 2 ? 2 : 1);
    w.casc_slot = max_entries * lb;
    w.F = 0;
    w.casc_a = align256(sizeof(float2) * (size_t)ncell * n_batch * lb);
    w.casc_b = w.casc_a + align256(sizeof(float) * (size_t)max_entries * lb * slots);
    w.smax = w.casc_b + align256(sizeof(float) * (size_t)max_entries * lb * slots);
    w.ebias = w.smax + align256(sizeof(float) * (size_t)n_batch * lb);
    w.flag = w.ebias + align256(sizeof(int32_t) * (size_t)n_batch * lb);
    w.total = w.flag + align256(sizeof(unsigned int));
    return w;
}

// Exact per-ray work on the host: number of segments the kernel's cell walk
// produces = plane crossings strictly inside the clipped interval + 1.
void count_work(rcx_plan* p)
{
    rcx_work& w = p->work;
    std::memset(&w, 0, sizeof(w));
    w.n_cascades = p->n_casc;
    w.top_skipped = p->top_skipped;
    const int32_t nx = p->grid.nx, nz = p->grid.nz;
    for (int32_t i = 0; i < p->n_casc; ++i) {
        const LevelDesc& L = p->levels[i];
        int64_t rays = level_entries(L), nonempty = 0, steps = 0;
        if (!(p->top_skipped && i == p->n_casc - 1)) {
            for (int32_t v = 0; v < L.pz; ++v)
                for (int32_t u = 0; u < L.px; ++u) {
                    const double cx = (u + 0.5) * L.s, cz = (v + 0.5) * L.s;
                    for (int32_t k = 0; k < L.nd; ++k) {
                        const double4 d = p->dirs_host[p->dir_off[i] + k];
                        double ax = (0.0 - cx) * d.z, bx = ((double)nx - cx) * d.z;
                        double az = (0.0 - cz) * d.w, bz = ((double)nz - cz) * d.w;
                        double lo = std::max(L.ta, std::max(std::min(ax, bx), std::min(az, bz)));
                        double hi = std::min(L.tb, std::min(std::max(ax, bx), std::max(az, bz)));
                        if (!(lo < hi)) continue;
                        ++nonempty;
                        double x0 = cx + lo * d.x, x1 = cx + hi * d.x;
                        double z0 = cz + lo * d.y, z1 = cz + hi * d.y;
                        int64_t nxc = d.x > 0 ? (int64_t)std::ceil(x1) - 1 - (int64_t)std::floor(x0)
                                              : (int64_t)std::ceil(x0) - 1 - (int64_t)std::floor(x1);
                        int64_t nzc = d.y > 0 ? (int64_t)std::ceil(z1) - 1 - (int64_t)std::floor(z0)
                                              : (int64_t)std::ceil(z0) - 1 - (int64_t)std::floor(z1);
                        steps += std::max<int64_t>(nxc, 0) + std::max<int64_t>(nzc, 0) + 1;
                    }
                }
        }
        // every flatland ray interval is marched once per inclination
        const int64_t ni = p->prm.n_incl;
        if (i < 16) {
            w.level_rays[i] = rays * ni;
            w.level_steps[i] = steps * ni;
        }
        w.rays_all += rays * ni;
        w.rays_nonempty += nonempty * ni;
        w.cell_steps += steps * ni;
    }
    p->work_done = true;
}


// Run `launch` between two recorded events when timing is enabled.
template <class F>
hipError_t timed(rcx_plan* p, int32_t level, hipStream_t st, F&& launch)
{
    if (level >= 0) ++p->n_march_enqueued;
    if (!p->timing) return launch();
    rcx_plan::Timed t{level, nullptr, nullptr};
    hipError_t e = hipEventCreate(&t.a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&t.b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(t.a);
        return e;
    }
    (void)hipEventRecord(t.a, st);
    e = launch();
    (void)hipEventRecord(t.b, st);
    p->pending.push_back(t);
    return e;
}

// The cascades of every batch, top-down (after the field preparation).
int32_t solve_batches(rcx_plan* p, int32_t n_wave, float* J, const WsLayout& w, char* ws, hipStream_t st)
{
    const int32_t nx = p->grid.nx, nz = p->grid.nz;
    const int64_t ncell = (int64_t)nx * nz;
    float2* F = (float2*)(ws + w.F);
    float* bufs[2] = {(float*)(ws + w.casc_a), (float*)(ws + w.casc_b)};
    const bool f16 = p->prm.storage == RCX_STORE_F16_SCALED;
    int32_t* ebias = (int32_t*)(ws + w.ebias);
    const int32_t lb = batch_width();
    const int32_t n_batch = (n_wave + lb - 1) / lb;
    const bool fuse_j = p->prm.c0_dirs == 4;
    if (p->prm.flags & RCX_FLAG_BILINEAR_FIX) {
        // bilinear fix: the cascades below the top trace each interval once
        // per bilinear probe; cascade 0 is stored, then averaged into J
        if (incl_slots(p)) {
            // the 8 inclinations as slots (one batch at a time)
            float sc[kInclSlots], wt[kInclSlots];
            for (int m = 0; m < kInclSlots; ++m) {
                sc[m] = (float)p->incl_scale[m];
                wt[m] = (float)p->incl_w[m];
            }
            for (int32_t b = 0; b < n_batch; ++b) {
                const float2* Fb = F + (size_t)b * ncell * lb;
                const int32_t nvalid = std::min(lb, n_wave - b * lb);
                int cur = 0;
                const void* up = nullptr;
                for (int32_t i = p->n_casc - 1; i >= 0; --i) {
                    if (p->top_skipped && i == p->n_casc - 1) continue;
                    const LevelDesc& L = p->levels[i];
                    CascIO io;
                    io.up = L.has_up ? up : nullptr;
                    io.up_f16 = false;
                    io.out = bufs[cur];
                    io.out_f16 = false;
                    io.ebias_b = ebias + (size_t)b * lb;
                    io.slot_stride = w.casc_slot;
                    const double4* dirs = p->dirs_dev + p->dir_off[i];
                    const bool fix = i + 1 < p->n_casc;
                    RCX_HIP_TRY(timed(p, i, st, [&] {
                        return fix ? launch_march_fix_incl(L, nx, nz, Fb, dirs, io, sc, st)
                                   : launch_march_merge_incl(L, nx, nz, Fb, dirs, io, sc, st);
                    }));
                    up = bufs[cur];
                    cur ^= 1;
                }
                RCX_HIP_TRY(timed(p, -1, st, [&] {
                    hipError_t e = hipSuccess;
                    for (int m = 0; m < kInclSlots && e == hipSuccess; ++m)
                        e = launch_j((const float*)up + m * w.casc_slot, J, b * lb, nvalid, ncell, p->prm.c0_dirs,
                                     wt[m], m > 0, st);
                    return e;
                }));
            }
            return ok();
        }
        // one pass per inclination (flatland: one pass); batches b and b+1
        // share the walks on the cascades with at most kPairMaxDirs
        // directions (as in the basic solve)
        for (int32_t m = 0; m < p->prm.n_incl; ++m) {
        const float jw = (float)p->incl_w[m];
        const bool jacc = m > 0;
        for (int32_t b = 0; b < n_batch;) {
            const bool pair = b + 1 < n_batch;
            const float2* Fb = F + (size_t)b * ncell * lb;
            const int32_t nvalid = std::min(lb, n_wave - b * lb);
            const int32_t nvalid1 = pair ? std::min(lb, n_wave - (b + 1) * lb) : 0;
            int cur = 0;
            const void* up = nullptr;
            bool up_f16 = false;
            for (int32_t i = p->n_casc - 1; i >= 0; --i) {
                if (p->top_skipped && i == p->n_casc - 1) continue;
                LevelDesc L = p->levels[i];
                L.ds_scale = p->incl_scale[m];
                CascIO io;
                io.up = L.has_up ? up : nullptr;
                io.up_f16 = up_f16;
                io.out = bufs[cur];
                io.out_f16 = f16 && i > 0;
                io.ebias_b = ebias + (size_t)b * lb;
                const bool together = pair && L.nd <= kPairMaxDirs;
                io.slot_stride = together ? w.casc_slot : 0;
                const bool fix = i + 1 < p->n_casc;
                const double4* dirs = p->dirs_dev + p->dir_off[i];
                RCX_HIP_TRY(timed(p, i, st, [&] {
                    return fix ? launch_march_fix(L, nx, nz, Fb, dirs, io, st)
                               : launch_march_merge(L, nx, nz, Fb, dirs, io, st);
                }));
                if (pair && !together) {
                    // batch b+1 into slot 1 (FP16 cascades: 2-byte elements)
                    CascIO io1 = io;
                    const size_t up_off = (size_t)w.casc_slot * (io.up_f16 ? (size_t)2 : sizeof(float));
                    const size_t out_off = (size_t)w.casc_slot * (io.out_f16 ? (size_t)2 : sizeof(float));
                    io1.up = io.up ? (const void*)((const char*)io.up + up_off) : nullptr;
                    io1.out = (void*)((char*)io.out + out_off);
                    io1.ebias_b = io.ebias_b + lb;
                    const float2* Fb1 = Fb + (size_t)ncell * lb;
                    RCX_HIP_TRY(timed(p, i, st, [&] {
                        return fix ? launch_march_fix(L, nx, nz, Fb1, dirs, io1, st)
                                   : launch_march_merge(L, nx, nz, Fb1, dirs, io1, st);
                    }));
                }
                up = bufs[cur];
                up_f16 = io.out_f16;
                cur ^= 1;
            }
            RCX_HIP_TRY(timed(p, -1, st, [&] {
                hipError_t e = launch_j((const float*)up, J, b * lb, nvalid, ncell, p->prm.c0_dirs, jw, jacc, st);
                if (e == hipSuccess && pair)
                    e = launch_j((const float*)up + w.casc_slot, J, (b + 1) * lb, nvalid1, ncell, p->prm.c0_dirs, jw,
                                 jacc, st);
                return e;
            }));
            b += pair ? 2 : 1;
        }
        }
        return ok();
    }
    if (incl_slots(p)) {
        // the inclinations as slots of each lane: J = sum_m w_m J_m formed in
        // the cascade-0 epilogue
        float sc[kInclSlots], wt[kInclSlots];
        for (int m = 0; m < kInclSlots; ++m) {
            sc[m] = (float)p->incl_scale[m];
            wt[m] = (float)p->incl_w[m];
        }
        for (int32_t b = 0; b < n_batch; ++b) {
            const float2* Fb = F + (size_t)b * ncell * lb;
            const int32_t nvalid = std::min(lb, n_wave - b * lb);
            int cur = 0;
            const void* up = nullptr;
            for (int32_t i = p->n_casc - 1; i >= 0; --i) {
                if (p->top_skipped && i == p->n_casc - 1) continue;
                const LevelDesc& L = p->levels[i];
                CascIO io;
                io.up = L.has_up ? up : nullptr;
                io.up_f16 = false;
                io.out = bufs[cur];
                io.out_f16 = false;
                io.ebias_b = ebias + (size_t)b * lb;
                io.slot_stride = w.casc_slot;
                if (i == 0 && fuse_j) {
                    RCX_HIP_TRY(timed(p, i, st, [&] {
                        return launch_march_merge_j_incl(L, nx, nz, Fb, p->dirs_dev + p->dir_off[i], io, J, b * lb,
                                                         nvalid, sc, wt, st);
                    }));
                    continue;
                }
                RCX_HIP_TRY(timed(p, i, st, [&] {
                    return launch_march_merge_incl(L, nx, nz, Fb, p->dirs_dev + p->dir_off[i], io, sc, st);
                }));
                up = bufs[cur];
                cur ^= 1;
            }
            if (!fuse_j) {
                RCX_HIP_TRY(timed(p, -1, st, [&] {
                    hipError_t e = hipSuccess;
                    for (int m = 0; m < kInclSlots && e == hipSuccess; ++m)
                        e = launch_j((const float*)up + m * w.casc_slot, J, b * lb, nvalid, ncell, p->prm.c0_dirs,
                                     wt[m], m > 0, st);
                    return e;
                }));
            }
        }
        return ok();
    }
    // one pass per inclination (Gauss-Radau in mu, the path length per
    // projected cell scaled by 1/sin): J = sum_m w_m J_m, written by the first
    // pass and accumulated by the others
    const int32_t n_incl = p->prm.n_incl;
    for (int32_t m = 0; m < n_incl; ++m) {
        const float jw = (float)p->incl_w[m];
        const bool jacc = m > 0;
        // batches b and b+1 marched together (one cell walk for 32 wavelengths)
        // on the cascades with at most kPairMaxDirs directions; the wider ones
        // (whose rays cross the most cells, and whose field reads rely on the
        // Infinity Cache holding one batch) march each batch alone into the
        // same two-slot layout. An odd last batch runs alone throughout.
        for (int32_t b = 0; b < n_batch;) {
            const bool pair = b + 1 < n_batch;
            const float2* Fb = F + (size_t)b * ncell * lb;
            const int32_t nvalid = std::min(lb, n_wave - b * lb);
            const int32_t nvalid1 = pair ? std::min(lb, n_wave - (b + 1) * lb) : 0;
            int cur = 0;
            const void* up = nullptr;
            bool up_f16 = false;
            for (int32_t i = p->n_casc - 1; i >= 0; --i) {
                if (p->top_skipped && i == p->n_casc - 1) continue;  // all rays empty: nothing to merge
                LevelDesc L = p->levels[i];
                L.ds_scale = p->incl_scale[m];
                CascIO io;
                io.up = L.has_up ? up : nullptr;
                io.up_f16 = up_f16;
                io.out = bufs[cur];
                io.out_f16 = f16 && i > 0;  // cascade 0 feeds J: kept in FP32
                io.ebias_b = ebias + (size_t)b * lb;
                const bool together = pair && L.nd <= kPairMaxDirs;
                io.slot_stride = together ? w.casc_slot : 0;
                if (i == 0 && fuse_j) {
                    // cascade 0 writes J directly (the 4 rows of a wavefront are
                    // the 4 directions of one cell); N_0 = 4: always together
                    RCX_HIP_TRY(timed(p, i, st, [&] {
                        return launch_march_merge_j(L, nx, nz, Fb, p->dirs_dev + p->dir_off[i], io, J, b * lb, nvalid,
                                                    nvalid1, jw, jacc, st);
                    }));
                    continue;
                }
                RCX_HIP_TRY(timed(p, i, st, [&] {
                    return launch_march_merge(L, nx, nz, Fb, p->dirs_dev + p->dir_off[i], io, st);
                }));
                if (pair && !together) {
                    // batch b+1 into slot 1 (FP16 cascades: 2-byte elements)
                    CascIO io1 = io;
                    const size_t up_off = (size_t)w.casc_slot * (io.up_f16 ? (size_t)2 : sizeof(float));
                    const size_t out_off = (size_t)w.casc_slot * (io.out_f16 ? (size_t)2 : sizeof(float));
                    io1.up = io.up ? (const void*)((const char*)io.up + up_off) : nullptr;
                    io1.out = (void*)((char*)io.out + out_off);
                    io1.ebias_b = io.ebias_b + lb;
                    RCX_HIP_TRY(timed(p, i, st, [&] {
                        return launch_march_merge(L, nx, nz, Fb + (size_t)ncell * lb, p->dirs_dev + p->dir_off[i], io1,
                                                  st);
                    }));
                }
                up = bufs[cur];
                up_f16 = io.out_f16;
                cur ^= 1;
            }
            if (!fuse_j) {
                RCX_HIP_TRY(timed(p, -1, st, [&] {
                    hipError_t e = launch_j((const float*)up, J, b * lb, nvalid, ncell, p->prm.c0_dirs, jw, jacc, st);
                    if (e == hipSuccess && pair)
                        e = launch_j((const float*)up + w.casc_slot, J, (b + 1) * lb, nvalid1, ncell, p->prm.c0_dirs, jw,
                                 jacc, st);
                    return e;
                }));
            }
            b += pair ? 2 : 1;
        }
    }
    return ok();
}


// The launches of one formal solve (after any input check).
int32_t enqueue_solve(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, float* J,
                             const WsLayout& w, char* ws, hipStream_t st)
{
    const int64_t ncell = (int64_t)p->grid.nx * p->grid.nz;
    float2* F = (float2*)(ws + w.F);
    if (p->timing) ++p->n_solves;
    const bool f16 = p->prm.storage == RCX_STORE_F16_SCALED;
    unsigned int* smax = (unsigned int*)(ws + w.smax);
    int32_t* ebias = (int32_t*)(ws + w.ebias);
    const int32_t lb = batch_width();
    const int32_t n_batch = (n_wave + lb - 1) / lb;
    if (p->mask_dev && p->levels[0].n_active == 0) {
        // sparse with nothing flagged: J = 0
        RCX_HIP_TRY(launch_mask_j(J, p->mask_dev, ncell, n_wave, st));
        return ok();
    }
    RCX_HIP_TRY(timed(p, -1, st, [&] {
        hipError_t e = launch_prep(chi, eta, F, n_wave, ncell, (float)p->grid.voxel_scale, f16 ? smax : nullptr, st);
        if (e == hipSuccess && f16) e = launch_ebias(n_batch * lb, smax, ebias, st);
        // sparse: unflagged cells transparent and empty (Sec. 3.5)
        if (e == hipSuccess && p->mask_dev) e = launch_mask_fields(F, p->mask_dev, ncell, n_batch, st);
        return e;
    }));
    const int32_t rc = solve_batches(p, n_wave, J, w, ws, st);
    if (rc != RCX_OK || !p->mask_dev) return rc;
    // sparse: J = 0 at unflagged cells
    RCX_HIP_TRY(timed(p, -1, st, [&] { return launch_mask_j(J, p->mask_dev, ncell, n_wave, st); }));
    return ok();
}

}  // namespace

extern "C" {

int32_t rcx_params_default(rcx_params* p)
{
    if (!p) return fail(RCX_E_INVALID, "rcx_params_default: null");
    p->n_cascades = 0;
    p->c0_dirs = 4;
    p->c0_t1 = 1.5;
    p->t_rule = RCX_T_GEOMETRIC;
    p->storage = RCX_STORE_F32;
    p->n_incl = 1;
    p->flags = 0;
    return ok();
}

int32_t rcx_plan_create(const rcx_grid* g, const rcx_params* prm, int32_t max_wave, rcx_plan** out)
{
    if (out) *out = nullptr;
    if (!g || !prm || !out) return fail(RCX_E_INVALID, "rcx_plan_create: null argument");
    if (g->nx <= 0 || g->nz <= 0 || max_wave <= 0)
        return fail(RCX_E_INVALID, "rcx_plan_create: nx, nz and max_wave must be positive");
    if (!(g->voxel_scale > 0.0)) return fail(RCX_E_INVALID, "rcx_plan_create: voxel_scale must be > 0");
    if ((int64_t)g->nx * g->nz > (int64_t(1) << 24))
        return fail(RCX_E_UNSUPPORTED, "rcx_plan_create: nx * nz must be at most 2^24 cells");
    if (prm->c0_dirs <= 0 || !(prm->c0_t1 > 0.0))
        return fail(RCX_E_INVALID, "rcx_plan_create: c0_dirs and c0_t1 must be positive");
    if (prm->t_rule != RCX_T_GEOMETRIC && prm->t_rule != RCX_T_LENGTH_X4)
        return fail(RCX_E_INVALID, "rcx_plan_create: unknown t_rule");
    if (prm->storage != RCX_STORE_F32 && prm->storage != RCX_STORE_F16_SCALED)
        return fail(RCX_E_UNSUPPORTED, "rcx_plan_create: unknown storage");
    if (prm->n_incl < 1 || prm->n_incl > 16)
        return fail(RCX_E_INVALID, "rcx_plan_create: n_incl must be in [1, 16] (1 = flatland)");
    if ((prm->flags & ~(RCX_FLAG_BILINEAR_FIX | RCX_FLAG_CHECK_INPUT)) != 0)
        return fail(RCX_E_INVALID, "rcx_plan_create: unknown flags");
    int32_t n_casc = prm->n_cascades == 0 ? auto_cascades(g->nx, g->nz) : prm->n_cascades;
    if (n_casc < 1 || n_casc > 16) return fail(RCX_E_INVALID, "rcx_plan_create: n_cascades must be in [1, 16]");
    if ((int64_t)prm->c0_dirs << (2 * (n_casc - 1)) > (int64_t(1) << 26))
        return fail(RCX_E_UNSUPPORTED, "rcx_plan_create: too many directions on the top cascade");

    rcx_plan* p = new (std::nothrow) rcx_plan();
    if (!p) return fail(RCX_E_NOMEM, "rcx_plan_create: host allocation");
    p->grid = *g;
    p->prm = *prm;
    p->prm.n_cascades = n_casc;
    p->max_wave = max_wave;
    p->n_casc = n_casc;
    {
        std::vector<double> mu;
        radau_nodes(prm->n_incl, mu, p->incl_w);
        p->incl_scale.resize(prm->n_incl);
        for (int32_t m = 0; m < prm->n_incl; ++m) p->incl_scale[m] = 1.0 / std::sqrt(1.0 - mu[m] * mu[m]);
    }
    p->levels.resize(n_casc);
    p->dir_off.resize(n_casc);
    int32_t off = 0;
    for (int32_t i = 0; i < n_casc; ++i) {
        LevelDesc& L = p->levels[i];
        const int32_t s = 1 << i;
        L.px = (g->nx + s - 1) / s;
        L.pz = (g->nz + s - 1) / s;
        L.nd = prm->c0_dirs << (2 * i);
        L.s = (double)s;
        L.ta = t_start(*prm, n_casc, i);
        L.tb = t_start(*prm, n_casc, i + 1);
        L.max_steps = g->nx + g->nz + 4;
        p->dir_off[i] = off;
        // Cone centres theta = 2 pi (k + 1/2) / N_i (children 4k..4k+3 nest).
        for (int32_t k = 0; k < L.nd; ++k) {
            const double th = 2.0 * M_PI * (k + 0.5) / (double)L.nd;
            const double wx = std::cos(th), wz = std::sin(th);
            p->dirs_host.push_back(make_double4(wx, wz, 1.0 / wx, 1.0 / wz));
        }
        off += L.nd;
    }
    for (int32_t i = 0; i < n_casc; ++i) {
        LevelDesc& L = p->levels[i];
        if (i + 1 < n_casc) {
            L.qx = p->levels[i + 1].px;
            L.qz = p->levels[i + 1].pz;
            L.nd_up = p->levels[i + 1].nd;
        }
    }
    const LevelDesc& top = p->levels[n_casc - 1];
    p->top_skipped = (n_casc > 1 && top.ta >= max_probe_corner_distance(*g, top)) ? 1 : 0;
    for (int32_t i = 0; i < n_casc; ++i) {
        LevelDesc& L = p->levels[i];
        L.has_up = (i + 1 < n_casc) && !(p->top_skipped && i + 1 == n_casc - 1);
        // long upper-cascade rays: run them in (4 x 4 probe tile x 32
        // direction wedge) groups, so the few groups one XCD holds at a time
        // cross a band of cells that fits its L2 (probe-major order spreads
        // them over full 360-degree fans)
        L.tile_p = 0;
        L.tile_d = 0;
        if (L.nd >= kTileMinDirs && L.nd % kTileDirs == 0) {
            L.tile_p = kTileProbes;
            L.tile_d = kTileDirs;
        }
    }

    hipError_t e = hipMalloc(&p->dirs_dev, sizeof(double4) * p->dirs_host.size());
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc(directions)");
    }
    e = hipMemcpy(p->dirs_dev, p->dirs_host.data(), sizeof(double4) * p->dirs_host.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        rcx_plan_destroy(p);
        return hip_fail(e, "hipMemcpy(directions)");
    }
    p->ws_own_bytes = ws_layout(p, max_wave).total;
    e = hipMalloc(&p->ws_own, p->ws_own_bytes);
    if (e != hipSuccess) {
        p->ws_own = nullptr;
        rcx_plan_destroy(p);
        return fail(RCX_E_NOMEM, std::string("rcx_plan_create: workspace hipMalloc: ") + hipGetErrorName(e));
    }
    // the allocation-free solve's scratch on this device (looked up once)
    const int32_t rc = scratch_address(&p->scratch);
    if (rc != RCX_OK) {
        rcx_plan_destroy(p);
        return rc;
    }
    *out = p;
    return ok();
}

int32_t rcx_formal_solve_noalloc(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, float* J,
                                 hipStream_t st)
{
    if (!p || !chi || !eta || !J) return fail(RCX_E_INVALID, "rcx_formal_solve_noalloc: null argument");
    if (n_wave <= 0 || n_wave > p->max_wave)
        return fail(RCX_E_INVALID, "rcx_formal_solve_noalloc: n_wave must be in [1, max_wave]");
    if (p->timing)
        return fail(RCX_E_INVALID, "rcx_formal_solve_noalloc: kernel timing creates events; disable it first");
    const size_t need = ws_layout(p, n_wave).total;
    if (need > kScratchBytes)
        return fail(RCX_E_WORKSPACE, "rcx_formal_solve_noalloc: the solve needs " + std::to_string(need) +
                                         " bytes of scratch, more than the library's " +
                                         std::to_string(kScratchBytes) + " (use rcx_formal_solve)");
    if (!p->scratch) return fail(RCX_E_HIP, "rcx_formal_solve_noalloc: no scratch address for the plan's device");
    return rcx_formal_solve(p, n_wave, chi, eta, J, p->scratch, kScratchBytes, st);
}

int32_t rcx_plan_set_active_host(rcx_plan* p, const uint8_t* active_host, int64_t* level_active_host)
{
    if (!p) return fail(RCX_E_INVALID, "rcx_plan_set_active_host: null plan");
    const int32_t nx = p->grid.nx, nz = p->grid.nz;
    // keep the flags: a change of launch order rebuilds the lists from them
    if (active_host && active_host != p->active_host.data())
        p->active_host.assign(active_host, active_host + (size_t)nx * nz);
    else if (!active_host)
        p->active_host.clear();
    // drop any previous flags: every probe active
    hipError_t e = hipSuccess;
    if (p->mask_dev) e = hipFree(p->mask_dev);
    if (p->plist_dev && e == hipSuccess) e = hipFree(p->plist_dev);
    p->mask_dev = nullptr;
    p->plist_dev = nullptr;
    for (auto& L : p->levels) {
        L.plist = nullptr;
        L.n_active = 0;
    }
    if (e != hipSuccess) return hip_fail(e, "rcx_plan_set_active_host: hipFree");
    if (!active_host) {
        if (level_active_host)
            for (int32_t i = 0; i < p->n_casc; ++i)
                level_active_host[i] = (int64_t)p->levels[i].px * p->levels[i].pz;
        return ok();
    }
    // flags: cascade 0 = the active cells; a probe of cascade i+1 is flagged
    // when it is one of the (clamped) bilinear taps of a flagged probe of
    // cascade i (Sec. 3.5)
    std::vector<std::vector<uint8_t>> flag(p->n_casc);
    flag[0].assign(active_host, active_host + (size_t)nx * nz);
    for (auto& f : flag[0]) f = f ? 1 : 0;
    for (int32_t i = 0; i + 1 < p->n_casc; ++i) {
        const LevelDesc& L = p->levels[i];
        const LevelDesc& U = p->levels[i + 1];
        flag[i + 1].assign((size_t)U.px * U.pz, 0);
        for (int32_t v = 0; v < L.pz; ++v)
            for (int32_t u = 0; u < L.px; ++u) {
                if (!flag[i][(size_t)v * L.px + u]) continue;
                const int bx0 = (u - 1) >> 1, bz0 = (v - 1) >> 1;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const int tx = std::min(std::max(bx0 + b, 0), U.px - 1);
                        const int tz = std::min(std::max(bz0 + a, 0), U.pz - 1);
                        flag[i + 1][(size_t)tz * U.px + tx] = 1;
                    }
            }
    }
    // lists in the launch order's probe order: tile by tile (row-major
    // tiles, row-major inside a tile) on tiled cascades, else probe-major
    std::vector<int32_t> all;
    std::vector<size_t> off(p->n_casc);
    std::vector<int32_t> cnt(p->n_casc);
    for (int32_t i = 0; i < p->n_casc; ++i) {
        const LevelDesc& L = p->levels[i];
        off[i] = all.size();
        if (L.tile_p <= 0) {
            for (int32_t q = 0; q < L.px * L.pz; ++q)
                if (flag[i][q]) all.push_back(q);
        } else {
            const int32_t tp = L.tile_p, ntx = (L.px + tp - 1) / tp, ntz = (L.pz + tp - 1) / tp;
            for (int32_t tz = 0; tz < ntz; ++tz)
                for (int32_t tx = 0; tx < ntx; ++tx)
                    for (int32_t j = 0; j < tp * tp; ++j) {
                        const int32_t u = tx * tp + j % tp, v = tz * tp + j / tp;
                        if (u < L.px && v < L.pz && flag[i][(size_t)v * L.px + u]) all.push_back(v * L.px + u);
                    }
        }
        cnt[i] = (int32_t)(all.size() - off[i]);
        if (level_active_host) level_active_host[i] = cnt[i];
    }
    e = hipMalloc(&p->mask_dev, (size_t)nx * nz);
    if (e == hipSuccess) e = hipMemcpy(p->mask_dev, flag[0].data(), (size_t)nx * nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->plist_dev, sizeof(int32_t) * std::max<size_t>(all.size(), 1));
    if (e == hipSuccess && !all.empty())
        e = hipMemcpy(p->plist_dev, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->mask_dev) (void)hipFree(p->mask_dev);
        if (p->plist_dev) (void)hipFree(p->plist_dev);
        p->mask_dev = nullptr;
        p->plist_dev = nullptr;
        return hip_fail(e, "rcx_plan_set_active_host");
    }
    for (int32_t i = 0; i < p->n_casc; ++i) {
        p->levels[i].plist = p->plist_dev + off[i];
        p->levels[i].n_active = cnt[i];
    }
    return ok();
}

int32_t rcx_plan_workspace_bytes(const rcx_plan* p, int32_t n_wave, size_t* bytes)
{
    if (!p || !bytes) return fail(RCX_E_INVALID, "rcx_plan_workspace_bytes: null argument");
    if (n_wave <= 0) return fail(RCX_E_INVALID, "rcx_plan_workspace_bytes: n_wave must be positive");
    *bytes = ws_layout(p, n_wave).total;
    return ok();
}

int32_t rcx_plan_work(rcx_plan* p, rcx_work* out)
{
    if (!p || !out) return fail(RCX_E_INVALID, "rcx_plan_work: null argument");
    if (!p->work_done) count_work(p);
    *out = p->work;
    return ok();
}

int32_t rcx_formal_solve(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, float* J,
                         void* workspace, size_t ws_bytes, hipStream_t st)
{
    if (!p || !chi || !eta || !J) return fail(RCX_E_INVALID, "rcx_formal_solve: null argument");
    if (n_wave <= 0 || n_wave > p->max_wave)
        return fail(RCX_E_INVALID, "rcx_formal_solve: n_wave must be in [1, max_wave]");
    const WsLayout w = ws_layout(p, n_wave);
    char* ws = (char*)workspace;
    if (!ws) {
        ws = (char*)p->ws_own;
    } else if (ws_bytes < w.total) {
        return fail(RCX_E_WORKSPACE, "rcx_formal_solve: workspace smaller than rcx_plan_workspace_bytes");
    }
    if (p->prm.flags & RCX_FLAG_CHECK_INPUT) {
        // chi and eta finite and non-negative (synchronises the stream)
        unsigned int* flag = (unsigned int*)(ws + w.flag);
        const int64_t n = (int64_t)n_wave * p->grid.nx * p->grid.nz;
        RCX_HIP_TRY(launch_zero_flag(flag, st));
        RCX_HIP_TRY(launch_check_f32(chi, n, kCheckNonNegative, flag, st));
        RCX_HIP_TRY(launch_check_f32(eta, n, kCheckNonNegative, flag, st));
        const int32_t rc = check_flag_result(flag, "rcx_formal_solve: chi or eta", st);
        if (rc != RCX_OK) return rc;
    }
    return enqueue_solve(p, n_wave, chi, eta, J, w, ws, st);
}

int32_t rcx_plan_set_timing(rcx_plan* p, int32_t enable)
{
    if (!p) return fail(RCX_E_INVALID, "rcx_plan_set_timing: null plan");
    p->timing = enable != 0;
    return ok();
}

int32_t rcx_plan_get_timing(rcx_plan* p, double* ms_level, double* ms_other, int64_t* n_launch,
                            int64_t* n_solves)
{
    if (!p || !ms_level || !ms_other || !n_launch || !n_solves)
        return fail(RCX_E_INVALID, "rcx_plan_get_timing: null argument");
    for (int32_t i = 0; i < p->n_casc; ++i) ms_level[i] = 0.0;
    *ms_other = 0.0;
    *n_launch = 0;
    int32_t rc = RCX_OK;
    for (auto& t : p->pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && rc == RCX_OK) rc = hip_fail(e, "rcx_plan_get_timing");
        if (t.level >= 0) {
            ms_level[t.level] += ms;
            ++*n_launch;
        } else {
            *ms_other += ms;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    p->pending.clear();
    *n_solves = p->n_solves;
    p->n_solves = 0;
    return rc == RCX_OK ? ok() : rc;
}

int32_t rcx_plan_set_order(rcx_plan* p, int32_t level, int32_t tile_p, int32_t tile_d, int32_t xcd_chunk,
                           int32_t shared_walk)
{
    if (!p || level < 0 || level >= p->n_casc) return fail(RCX_E_INVALID, "rcx_plan_set_order: bad plan or level");
    LevelDesc& L = p->levels[level];
    if (tile_p < 0 || tile_p > 64 || xcd_chunk < 1 || xcd_chunk > (1 << 16) || (shared_walk != 0 && shared_walk != 1))
        return fail(RCX_E_INVALID,
                    "rcx_plan_set_order: tile_p must be in [0, 64], xcd_chunk in [1, 65536], shared_walk 0 or 1");
    if (tile_p > 0 && (tile_d < 4 || tile_d % 4 != 0 || L.nd % tile_d != 0))
        return fail(RCX_E_INVALID, "rcx_plan_set_order: tile_d must be a multiple of 4 dividing the directions");
    L.tile_p = tile_p;
    L.tile_d = tile_p > 0 ? tile_d : 0;
    L.xcd_chunk = xcd_chunk;
    L.shared_walk = shared_walk;
    if (p->mask_dev) {
        // the flagged-probe lists follow the launch order: rebuild them
        const std::vector<uint8_t> flags = p->active_host;
        return rcx_plan_set_active_host(p, flags.data(), nullptr);
    }
    return ok();
}

int32_t rcx_plan_get_order(const rcx_plan* p, int32_t level, int32_t* order4_host)
{
    if (!p || !order4_host || level < 0 || level >= p->n_casc)
        return fail(RCX_E_INVALID, "rcx_plan_get_order: bad argument");
    const LevelDesc& L = p->levels[level];
    order4_host[0] = L.tile_p;
    order4_host[1] = L.tile_d;
    order4_host[2] = L.xcd_chunk;
    order4_host[3] = L.shared_walk;
    return ok();
}

int32_t rcx_autotune(rcx_plan* p, const char* cache_path, hipStream_t st)
{
    if (!p) return fail(RCX_E_INVALID, "rcx_autotune: null plan");
    const int32_t nx = p->grid.nx, nz = p->grid.nz;
    const int64_t ncell = (int64_t)nx * nz;
    const int32_t n_wave = std::min(p->max_wave, 2 * batch_width());
    std::vector<int32_t> tun;  // the cascades whose launch order is tuned
    for (int32_t i = 0; i < p->n_casc; ++i)
        if (p->levels[i].nd >= kTileMinDirs && !(p->top_skipped && i == p->n_casc - 1)) tun.push_back(i);
    if (tun.empty()) return ok();
    int dev = 0;
    RCX_HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    RCX_HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::ostringstream key;
    key << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu/" << nx << "x" << nz << "/c" << p->n_casc
        << "/d" << p->prm.c0_dirs << "/t1=" << p->prm.c0_t1 << "/r" << p->prm.t_rule << "/s" << p->prm.storage
        << "/i" << p->prm.n_incl << "/f" << (p->prm.flags & RCX_FLAG_BILINEAR_FIX) << "/w" << n_wave
        << "/walk2";  // orders with the walk mode (a fifth field)
    if (p->mask_dev) key << "/sparse" << p->levels[0].n_active;
    const std::string k = key.str();
    const std::string pre = "{\"key\": \"" + k + "\", \"orders\": \"";
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            if (line.compare(0, pre.size(), pre) != 0) continue;
            // "level:tile_p:tile_d:chunk:walk,..." up to the closing quote
            std::istringstream in(line.substr(pre.size(), line.find('"', pre.size()) - pre.size()));
            std::string item;
            int32_t rc = RCX_OK;
            while (rc == RCX_OK && std::getline(in, item, ',')) {
                int lv = -1, tp = 0, td = 0, ch = 0, sw = 0;
                if (std::sscanf(item.c_str(), "%d:%d:%d:%d:%d", &lv, &tp, &td, &ch, &sw) == 5)
                    rc = rcx_plan_set_order(p, lv, tp, td, ch, sw);
            }
            return rc;
        }
    }
    // time candidate orders on uniform fields (the march's work and memory
    // traffic do not depend on the values)
    struct Cand {
        int32_t tp, td, ch, sw;
    };
    // the shared walk serves the basic march of a dense plan with one
    // inclination (with the bilinear fix, only its top marched cascade);
    // elsewhere its setting changes nothing and is kept 0
    auto walk_applies = [p](int32_t i) {
        return !p->mask_dev && p->prm.n_incl == 1 &&
               (!(p->prm.flags & RCX_FLAG_BILINEAR_FIX) || !p->levels[i].has_up);
    };
    bool walk_cands = false;
    for (int32_t i : tun) walk_cands = walk_cands || walk_applies(i);
    std::vector<Cand> cands;
    for (int32_t ch : {32, 128, 512}) {
        cands.push_back({0, 0, ch, 0});
        for (int32_t tp : {2, 4, 8})
            for (int32_t td : {16, 32, 64})
                for (int32_t sw : {0, 1})
                    if (sw == 0 || walk_cands) cands.push_back({tp, td, ch, sw});
    }
    std::vector<LevelDesc> saved = p->levels;
    const bool timing = p->timing;
    float* buf = nullptr;
    void* ws = nullptr;
    const size_t nfield = (size_t)n_wave * ncell;
    hipError_t e = hipMalloc(&buf, sizeof(float) * 3 * nfield);
    const size_t ws_bytes = ws_layout(p, n_wave).total;
    if (e == hipSuccess && !p->ws_own) e = hipMalloc(&ws, ws_bytes);
    if (e != hipSuccess) {
        if (buf) (void)hipFree(buf);
        return fail(RCX_E_NOMEM, "rcx_autotune: temporary fields");
    }
    int32_t rc = RCX_OK;
    e = launch_fill_f32(buf, (int64_t)2 * nfield, 1.0f, st);
    std::vector<std::vector<double>> ms(cands.size(), std::vector<double>(p->n_casc, 0.0));
    std::vector<double> lvl(p->n_casc);
    double other = 0.0;
    int64_t nl = 0, ns = 0;
    for (size_t c = 0; c < cands.size() && rc == RCX_OK && e == hipSuccess; ++c) {
        for (int32_t i : tun) {
            const int32_t td = cands[c].tp > 0 && p->levels[i].nd % cands[c].td != 0 ? 4 : cands[c].td;
            rc = rcx_plan_set_order(p, i, cands[c].tp, td, cands[c].ch, walk_applies(i) ? cands[c].sw : 0);
            if (rc != RCX_OK) break;
        }
        if (rc != RCX_OK) break;
        p->timing = false;
        rc = rcx_formal_solve(p, n_wave, buf, buf + nfield, buf + 2 * nfield, ws, ws_bytes, st);
        if (rc != RCX_OK) break;
        p->timing = true;
        for (int r = 0; r < 2 && rc == RCX_OK; ++r)
            rc = rcx_formal_solve(p, n_wave, buf, buf + nfield, buf + 2 * nfield, ws, ws_bytes, st);
        if (rc == RCX_OK) rc = rcx_plan_get_timing(p, lvl.data(), &other, &nl, &ns);
        ms[c] = lvl;
    }
    p->timing = timing;
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (ws) (void)hipFree(ws);
    if (e != hipSuccess && rc == RCX_OK) rc = hip_fail(e, "rcx_autotune");
    if (rc != RCX_OK) {
        p->levels = saved;
        if (p->mask_dev) {
            const std::vector<uint8_t> flags = p->active_host;
            (void)rcx_plan_set_active_host(p, flags.data(), nullptr);
        }
        return rc;
    }
    std::ostringstream orders, times;
    for (size_t q = 0; q < tun.size(); ++q) {
        const int32_t i = tun[q];
        size_t best = 0;
        for (size_t c = 1; c < cands.size(); ++c)
            if (ms[c][i] < ms[best][i]) best = c;
        const int32_t td = cands[best].tp > 0 && p->levels[i].nd % cands[best].td != 0 ? 4 : cands[best].td;
        const int32_t sw = walk_applies(i) ? cands[best].sw : 0;
        rc = rcx_plan_set_order(p, i, cands[best].tp, td, cands[best].ch, sw);
        if (rc != RCX_OK) return rc;
        orders << (q ? "," : "") << i << ":" << cands[best].tp << ":" << p->levels[i].tile_d << ":" << cands[best].ch
               << ":" << sw;
        times << (q ? "," : "") << i << ":" << ms[best][i] / 2.0 << "/" << ms[0][i] / 2.0;
    }
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << pre << orders.str() << "\", \"ms_best_vs_first\": \"" << times.str() << "\"}\n";
    }
    return ok();
}

int32_t rcx_plan_destroy(rcx_plan* p)
{
    if (!p) return ok();
    for (auto& t : p->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    if (p->dirs_dev) (void)hipFree(p->dirs_dev);
    if (p->ws_own) (void)hipFree(p->ws_own);
    if (p->mask_dev) (void)hipFree(p->mask_dev);
    if (p->plist_dev) (void)hipFree(p->plist_dev);
    delete p;
    return ok();
}

const char* rcx_error_string(int32_t code)
{
    switch (code) {
    case RCX_OK: return "ok";
    case RCX_W_NOT_CONVERGED: return "not converged within the iteration limit";
    case RCX_E_INVALID: return "invalid argument";
    case RCX_E_UNSUPPORTED: return "unsupported configuration";
    case RCX_E_NOMEM: return "out of memory";
    case RCX_E_HIP: return "HIP runtime error";
    case RCX_E_WORKSPACE: return "workspace too small";
    case RCX_E_NONFINITE: return "input value not finite or out of range";
    default: return "unknown status code";
    }
}

int32_t rcx_last_error(char* buf, size_t n)
{
    if (buf && n > 0) std::snprintf(buf, n, "%s", g_last_msg);
    return g_last_code;
}

}  // extern "C"

namespace rcx {
int32_t plan_enqueue_solve(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, float* J,
                           hipStream_t st, int64_t* march_launches)
{
    if (!p || !p->ws_own || n_wave <= 0 || n_wave > p->max_wave)
        return fail(RCX_E_INVALID, "plan_enqueue_solve: no own workspace or n_wave outside [1, max_wave]");
    p->n_march_enqueued = 0;
    const int32_t rc = enqueue_solve(p, n_wave, chi, eta, J, ws_layout(p, n_wave), (char*)p->ws_own, st);
    if (march_launches) *march_launches = p->n_march_enqueued;
    return rc;
}
}  // namespace rcx

