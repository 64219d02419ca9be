// emergent.hip -- emergent intensity along parallel long characteristics
// (Osborne & Sannikov, arXiv:2408.14425, Sec. 3.9: a single-pass long
// characteristics solver for rays of any direction through the domain,
// traced front to back from the point where the emergent intensity is
// wanted).
//
// A beam of n_rays parallel rays of light direction w, one cell apart
// across the beam and centred on the domain, is traced from outside the
// domain back along -w with the same cooperative FP64 cell walk and FP32
// front-to-back update as the cascade march (4 rays x 16 wavelengths per
// wavefront); what has accumulated when a ray leaves the far side is the
// intensity emerging towards the observer.
#include "march_rows.h"

#include <cmath>

namespace rcx {
namespace {

using march::kBlock;
using march::kLB;
using march::kRaysPerBlock;

// I[lam0 + l][j] for the rays j of the beam: origin o0 + s_j p, s_j = j +
// 1/2 - n_rays/2 (cells across the beam), direction d = -w.
__global__ __launch_bounds__(kBlock) void k_emergent(LevelDesc L, int32_t nx, int32_t nz, march::FieldOp op,
                                                     double ox0, double oz0, double px, double pz, double4 d,
                                                     int32_t n_rays, float* __restrict__ out, int32_t lam0,
                                                     int32_t n_valid)
{
    __shared__ uint4 seg[kBlock / 64][4][march::kSegRow];
    __shared__ march::FieldOp::Stage stg[1][4][march::kStgRow];
    const march::RowCtx c = march::row_ctx();
    op.init(c.l);
    seg[c.w][c.row][c.l] = make_uint4(0u, 0u, 0u, 0u);
    march::wave_sync();
    const int64_t stride = (int64_t)gridDim.x * kRaysPerBlock;
    for (int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + c.w) * 4; base < n_rays; base += stride) {
        const int64_t j = base + c.row;
        const bool active = j < n_rays;
        const double s = (double)(active ? j : 0) + 0.5 - 0.5 * (double)n_rays;
        float I[1], T[1];
        march::walk_ray(L, nx, nz, op, ox0 + s * px, oz0 + s * pz, d, 0.0, INFINITY, active, seg[c.w], stg[0], c,
                        I, T);
        if (active && c.l < n_valid) out[(int64_t)(lam0 + c.l) * n_rays + j] = I[0];
    }
}

}  // namespace
}  // namespace rcx

using namespace rcx;

extern "C" int32_t rcx_emergent(rcx_plan* p, int32_t n_wave, const float* chi, const float* eta, double wx,
                                double wz, int32_t n_rays, float* I, hipStream_t st)
{
    if (!p || !chi || !eta || !I) return fail(RCX_E_INVALID, "rcx_emergent: null argument");
    if (n_wave <= 0 || n_wave > p->max_wave) return fail(RCX_E_INVALID, "rcx_emergent: n_wave must be in [1, max_wave]");
    if (n_rays <= 0) return fail(RCX_E_INVALID, "rcx_emergent: n_rays must be positive");
    const double wn = std::hypot(wx, wz);
    if (!(wn > 0.0) || !std::isfinite(wn)) return fail(RCX_E_INVALID, "rcx_emergent: direction must be non-zero");
    wx /= wn;
    wz /= wn;
    const int32_t nx = p->grid.nx, nz = p->grid.nz;
    const int64_t ncell = (int64_t)nx * nz;
    const int32_t n_batch = (n_wave + kLB - 1) / kLB;
    // the field batches at the start of the plan's own workspace (sized for
    // max_wave wavelengths)
    float2* F = (float2*)p->ws_own;
    if (p->prm.flags & RCX_FLAG_CHECK_INPUT) {
        // the flag word after the field batches of n_wave wavelengths (the
        // workspace holds at least that much)
        unsigned int* flag = (unsigned int*)((char*)p->ws_own + sizeof(float2) * (size_t)ncell * n_batch * kLB);
        RCX_HIP_TRY(launch_zero_flag(flag, st));
        RCX_HIP_TRY(launch_check_f32(chi, (int64_t)n_wave * ncell, kCheckNonNegative, flag, st));
        RCX_HIP_TRY(launch_check_f32(eta, (int64_t)n_wave * ncell, kCheckNonNegative, flag, st));
        const int32_t rc = check_flag_result(flag, "rcx_emergent: chi or eta", st);
        if (rc != RCX_OK) return rc;
    }
    RCX_HIP_TRY(launch_prep(chi, eta, F, n_wave, ncell, (float)p->grid.voxel_scale, nullptr, st));
    if (p->mask_dev) RCX_HIP_TRY(launch_mask_fields(F, p->mask_dev, ncell, n_batch, st));
    // beam: centred on the domain, starting outside it on the observer's
    // side; march direction -w (an axis-parallel ray gets a 1e-12 minor
    // component so its plane steps stay finite; its cells are unchanged)
    const double R = 0.5 * std::hypot((double)nx, (double)nz) + 2.0;
    const double ox0 = 0.5 * nx + R * wx, oz0 = 0.5 * nz + R * wz;
    double dx = -wx, dz = -wz;
    if (std::fabs(dx) < 1e-12) dx = dx < 0.0 ? -1e-12 : 1e-12;
    if (std::fabs(dz) < 1e-12) dz = dz < 0.0 ? -1e-12 : 1e-12;
    const double4 d = make_double4(dx, dz, 1.0 / dx, 1.0 / dz);
    LevelDesc L{};
    L.ds_scale = 1.0;
    const uint32_t fb_bytes = (uint32_t)(ncell * kLB * sizeof(float2));
    for (int32_t b = 0; b < n_batch; ++b) {
        march::FieldOp op{};
        op.Fb = F + (size_t)b * ncell * kLB;
        op.fb_bytes = fb_bytes;
        const int32_t n_valid = std::min(kLB, n_wave - b * kLB);
        hipLaunchKernelGGL(k_emergent, march_grid(n_rays), dim3(kBlock), 0, st, L, nx, nz, op, ox0, oz0, -wz, wx, d,
                           n_rays, I, b * kLB, n_valid);
        RCX_HIP_TRY(hipGetLastError());
    }
    return RCX_OK;
}
