// fs_kernels.hip -- gfx950 kernels of the radiance-cascades formal solution
// (Osborne & Sannikov, arXiv:2408.14425, Secs. 2.2-2.3 and 3.2).
//
// Input preparation and J for the GivenFs formal solution; the march itself
// is the template in march_rows.h.
//
// Wavelengths are processed in batches of 16 (kLB). Data layout in HBM, with
// c = z * nx + x the cell index and l the wavelength within a batch:
//   F       [batch][c][16]          float2 {chi * voxel * log2(e) (floored), S = eta/chi}
//   cascade [slot][(p * N_i + k)][16] float merged radiance of probe p, direction k;
//                                   slot 1 = the second batch of a pair, slots 0-7
//                                   = the inclinations, a fixed stride apart
//   J       [lambda][c]             float  (the caller's layout)
// A batch of F is 128 MB at 1024^2 (half the 256 MB Infinity Cache); the
// cascades of a batch (or of a pair of batches) are marched top-down before
// the next batch starts.
#include "march_rows.h"

#include <algorithm>
#include <type_traits>
#include <cmath>

namespace rcx {

namespace {

using march::kBlock;
using march::kLB;
using march::kLog2e;

constexpr float kChiFloor = 1e-20f;  // per cell, natural units

// ---------------------------------------------------------------- prep
// chi, eta [n_wave][ncell] -> F [batch][ncell][16], one 64-cell x 16-wavelength
// tile per block through LDS. Wavelengths past n_wave are padded with
// {1, 0} (no emission).
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ chi,
                                              const float* __restrict__ eta,
                                              float2* __restrict__ F, int32_t n_wave,
                                              int64_t ncell, float voxel, unsigned int* __restrict__ smax_bits)
{
    __shared__ float2 tile[kLB][65];
    __shared__ float smax[kLB];
    if (threadIdx.x < kLB) smax[threadIdx.x] = 0.0f;
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int32_t b = blockIdx.y;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = (t >> 6) + 4 * r;
        const int cc = t & 63;
        const int32_t lam = b * kLB + l;
        const int64_t c = c0 + cc;
        float2 v = make_float2(1.0f, 0.0f);
        if (lam < n_wave && c < ncell) {
            const float ch = chi[(int64_t)lam * ncell + c];
            const float et = eta[(int64_t)lam * ncell + c];
            const float cv = ch * voxel;
            v = (cv >= kChiFloor) ? make_float2(cv * kLog2e, et / ch)
                                  : make_float2(kChiFloor * kLog2e, et * voxel / kChiFloor);
        }
        tile[l][cc] = v;
    }
    __syncthreads();
    if (smax_bits) {  // per-wavelength maximum of S over this tile (S >= 0: float bits order as integers)
        if (threadIdx.x < kLB) {
            float m = 0.0f;
            for (int cc = 0; cc < 64; ++cc) m = fmaxf(m, tile[threadIdx.x][cc].y);
            atomicMax(&smax_bits[b * kLB + threadIdx.x], __float_as_uint(m));
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = t & 15;
        const int cc = (t >> 4) + 16 * r;
        const int64_t c = c0 + cc;
        if (c < ncell) F[((int64_t)b * ncell + c) * kLB + l] = tile[l][cc];
    }
}

// Per-wavelength exponent bias of the 16-bit cascade storage: the FP32
// exponent field of max S less 62, so the codes cover 2 max S downwards
// (march_rows.h, enc_h16). max S is non-negative and finite.
__global__ void k_ebias(int32_t n, const unsigned int* __restrict__ smax_bits, int32_t* __restrict__ ebias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ebias[i] = (int32_t)((smax_bits[i] & 0x7FFFFFFFu) >> 23) - 62;
}

// Input check (RCX_FLAG_CHECK_INPUT): *flag |= 1 if a value is not finite,
// 2 if a finite value is out of range: below 0 (range kNonNegative), not
// above 0 (kPositive), never (kFinite). One atomic per wavefront.
template <class T>
__global__ void k_check_values(const T* __restrict__ a, int64_t n, int32_t range, unsigned int* __restrict__ flag)
{
    unsigned int bits = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = a[i];
        if (!isfinite(v))
            bits |= 1u;
        else if ((range == kCheckNonNegative && v < T(0)) || (range == kCheckPositive && !(v > T(0))))
            bits |= 2u;
    }
    const unsigned int any1 = __ballot(bits & 1u) != 0ull ? 1u : 0u;
    const unsigned int any2 = __ballot(bits & 2u) != 0ull ? 2u : 0u;
    if ((threadIdx.x & 63) == 0 && (any1 | any2)) atomicOr(flag, any1 | any2);
}

__global__ void k_fill_f32(float* p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(unsigned int* p, int32_t n, unsigned int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Sparse solve: cells with mask 0 are transparent and emit nothing
// (F = {0, 0} in every batch), and their J is 0. Grid-stride over
// (batch or wavelength) x cell; F is written as 16 float2 per cell.
__global__ __launch_bounds__(256) void k_mask_fields(float2* __restrict__ F, const uint8_t* __restrict__ mask,
                                                     int64_t ncell, int32_t n_batch)
{
    const int64_t n = (int64_t)n_batch * ncell * kLB;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = (i / kLB) % ncell;
        if (!mask[c]) F[i] = make_float2(0.0f, 0.0f);
    }
}

__global__ __launch_bounds__(256) void k_mask_j(float* __restrict__ J, const uint8_t* __restrict__ mask, int64_t ncell,
                                                int32_t n_wave)
{
    const int64_t n = (int64_t)n_wave * ncell;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!mask[i % ncell]) J[i] = 0.0f;
}

// ---------------------------------------------------------------- J
// J[lam0 + l][c] = (1/N_0) sum_k Itilde_0[(c * N_0 + k)][l] for one batch,
// through a 64-cell x 16-wavelength LDS tile.
__global__ __launch_bounds__(256) void k_j(const float* __restrict__ I0, float* __restrict__ J,
                                           int32_t lam0, int32_t n_valid, int64_t ncell, int32_t n0, float w,
                                           int32_t acc_j)
{
    __shared__ float tile[kLB][65];
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const float inv = w / (float)n0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = t & 15;
        const int cc = (t >> 4) + 16 * r;
        const int64_t c = c0 + cc;
        float acc = 0.0f;
        if (c < ncell)
            for (int k = 0; k < n0; ++k) acc += I0[(c * n0 + k) * kLB + l];
        tile[l][cc] = acc * inv;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = (t >> 6) + 4 * r;
        const int cc = t & 63;
        const int64_t c = c0 + cc;
        if (l < n_valid && c < ncell) {
            float* j = &J[(int64_t)(lam0 + l) * ncell + c];
            *j = acc_j ? *j + tile[l][cc] : tile[l][cc];
        }
    }
}

}  // namespace

int32_t batch_width() { return kLB; }

dim3 march_grid(int64_t rays)
{
    int64_t blocks = (rays + march::kRaysPerBlock - 1) / march::kRaysPerBlock;
    const int64_t cap = 1 << 20;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return dim3((unsigned)blocks);
}

hipError_t launch_prep(const float* chi, const float* eta, float2* F, int32_t n_wave, int64_t ncell,
                       float voxel, unsigned int* smax_bits, hipStream_t st)
{
    const int32_t nb = (n_wave + kLB - 1) / kLB;
    if (smax_bits) {
        hipLaunchKernelGGL(k_fill_u32, dim3((nb * kLB + 255) / 256), dim3(256), 0, st, smax_bits, nb * kLB, 0u);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)((ncell + 63) / 64), (unsigned)nb);
    hipLaunchKernelGGL(k_prep, grid, dim3(256), 0, st, chi, eta, F, n_wave, ncell, voxel, smax_bits);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st)
{
    const int64_t blocks = std::max<int64_t>(std::min<int64_t>((n + 255) / 256, 16384), 1);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero_flag(unsigned int* flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, flag, 1, 0u);
    return hipGetLastError();
}

hipError_t launch_check_f32(const float* a, int64_t n, int32_t range, unsigned int* flag, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_check_values<float>, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, a, n,
                       range, flag);
    return hipGetLastError();
}

hipError_t launch_check_f64(const double* a, int64_t n, int32_t range, unsigned int* flag, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_check_values<double>, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, a, n,
                       range, flag);
    return hipGetLastError();
}

hipError_t launch_ebias(int32_t n, const unsigned int* smax_bits, int32_t* ebias, hipStream_t st)
{
    hipLaunchKernelGGL(k_ebias, dim3((n + 255) / 256), dim3(256), 0, st, n, smax_bits, ebias);
    return hipGetLastError();
}

namespace {
template <class Op, class Epi, class Up>
hipError_t launch_fs(const LevelDesc& L0, int32_t nx, int32_t nz, const Op& op, const Epi& epi, const double4* dirs,
                     const Up& up, hipStream_t st)
{
    LevelDesc L = L0;
    // dense tiled orders of the field ops with an even tile and whole-cell
    // probe spacing run the 4 rows of a wavefront on one direction and
    // share its cell walk (bitwise the same results); the J epilogues sum
    // the 4 rows as the 4 directions of one probe and keep the row walk
    constexpr bool kShareable =
        (std::is_same<Op, march::FieldOp>::value || std::is_same<Op, march::FieldOp2>::value) &&
        !std::is_same<Epi, march::JEpi>::value && !std::is_same<Epi, march::JEpi2>::value;
    const bool shared =
        kShareable && L.shared_walk && L.tile_p > 0 && L.tile_p % 2 == 0 && !L.plist && L.s == std::floor(L.s);
    if (!set_decode(L)) return hipErrorInvalidValue;  // more rays than 31-bit indices
    const int64_t total = level_launch_rays(L);
    if constexpr (kShareable) {
        if (shared) {
            hipLaunchKernelGGL((march::k_march_shared<Op, Epi, Up>), march_grid(total), dim3(kBlock), 0, st, L, nx, nz,
                               op, epi, dirs, up, total);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((march::k_march_rows<Op, Epi, Up>), march_grid(total), dim3(kBlock), 0, st, L, nx, nz, op, epi,
                       dirs, up, total);
    return hipGetLastError();
}

// The reader of the cascade above, then the launch with it.
template <class Op, class Epi>
hipError_t launch_fs_up(const LevelDesc& L, int32_t nx, int32_t nz, const Op& op, const Epi& epi,
                        const double4* dirs, const CascIO& io, hipStream_t st)
{
    if (!io.up_f16) {
        march::UpF32 up{(const float*)io.up};
        up.stride = io.slot_stride;
        return launch_fs(L, nx, nz, op, epi, dirs, up, st);
    }
    march::UpF16 up{(const uint16_t*)io.up, io.ebias_b};
    up.stride = io.slot_stride;
    return launch_fs(L, nx, nz, op, epi, dirs, up, st);
}

// The bilinear-fix kernel: one interval per wavefront, so 4 x the
// intervals' rows.
template <class Op, class Epi, class Up>
hipError_t launch_fix_k(const LevelDesc& L0, int32_t nx, int32_t nz, const Op& op, const Epi& epi, const double4* dirs,
                        const Up& up, hipStream_t st)
{
    LevelDesc L = L0;
    if (!set_decode(L)) return hipErrorInvalidValue;  // more rays than 31-bit indices
    const int64_t total = level_launch_rays(L);
    hipLaunchKernelGGL((march::k_march_fix<Op, Epi, Up>), march_grid(4 * total), dim3(kBlock), 0, st, L, nx, nz, op,
                       epi, dirs, up, total);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_march_fix(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                            const CascIO& io, hipStream_t st)
{
    const uint32_t fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    if (io.slot_stride != 0) {
        // two batches per lane (slot 1 io.slot_stride elements on)
        march::FieldOp2 op{};
        op.Fb = Fb;
        op.fb_bytes = fb_bytes;
        if (!io.up_f16) {
            march::UpF32 up{(const float*)io.up};
            up.stride = io.slot_stride;
            if (!io.out_f16)
                return launch_fix_k(L, nx, nz, op, march::StoreEpi2{(float*)io.out, io.slot_stride}, dirs, up, st);
            return launch_fix_k(L, nx, nz, op,
                                march::StoreF16Epi2{(uint16_t*)io.out, io.slot_stride, io.ebias_b}, dirs,
                                up, st);
        }
        march::UpF16 up{(const uint16_t*)io.up, io.ebias_b};
        up.stride = io.slot_stride;
        if (!io.out_f16)
            return launch_fix_k(L, nx, nz, op, march::StoreEpi2{(float*)io.out, io.slot_stride}, dirs, up, st);
        return launch_fix_k(L, nx, nz, op, march::StoreF16Epi2{(uint16_t*)io.out, io.slot_stride, io.ebias_b},
                            dirs, up, st);
    }
    march::FieldOp op{};
    op.Fb = Fb;
    op.fb_bytes = fb_bytes;
    if (!io.up_f16) {
        const march::UpF32 up{(const float*)io.up};
        if (!io.out_f16) return launch_fix_k(L, nx, nz, op, march::StoreEpi{(float*)io.out}, dirs, up, st);
        return launch_fix_k(L, nx, nz, op, march::StoreF16Epi{(uint16_t*)io.out, io.ebias_b}, dirs, up, st);
    }
    march::UpF16 up{(const uint16_t*)io.up, io.ebias_b};
    if (!io.out_f16) return launch_fix_k(L, nx, nz, op, march::StoreEpi{(float*)io.out}, dirs, up, st);
    return launch_fix_k(L, nx, nz, op, march::StoreF16Epi{(uint16_t*)io.out, io.ebias_b}, dirs, up, st);
}

hipError_t launch_march_merge(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                              const CascIO& io, hipStream_t st)
{
    const uint32_t fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    if (io.slot_stride != 0) {
        march::FieldOp2 op{};
        op.Fb = Fb;
        op.fb_bytes = fb_bytes;
        if (!io.out_f16) return launch_fs_up(L, nx, nz, op, march::StoreEpi2{(float*)io.out, io.slot_stride}, dirs, io, st);
        return launch_fs_up(L, nx, nz, op, march::StoreF16Epi2{(uint16_t*)io.out, io.slot_stride, io.ebias_b},
                            dirs, io, st);
    }
    march::FieldOp op{};
    op.Fb = Fb;
    op.fb_bytes = fb_bytes;
    if (!io.out_f16) return launch_fs_up(L, nx, nz, op, march::StoreEpi{(float*)io.out}, dirs, io, st);
    return launch_fs_up(L, nx, nz, op, march::StoreF16Epi{(uint16_t*)io.out, io.ebias_b}, dirs, io, st);
}

hipError_t launch_march_merge_j(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                const CascIO& io, float* J, int32_t lam0, int32_t n_valid, int32_t n_valid1,
                                float w, bool acc, hipStream_t st)
{
    const uint32_t fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    if (io.slot_stride != 0) {
        march::FieldOp2 op{};
        op.Fb = Fb;
        op.fb_bytes = fb_bytes;
        return launch_fs_up(L, nx, nz, op, march::JEpi2{J, lam0, n_valid, n_valid1, (int64_t)nx * nz, w, acc}, dirs,
                            io, st);
    }
    march::FieldOp op{};
    op.Fb = Fb;
    op.fb_bytes = fb_bytes;
    return launch_fs_up(L, nx, nz, op, march::JEpi{J, lam0, n_valid, (int64_t)nx * nz, w, acc}, dirs, io, st);
}

hipError_t launch_march_merge_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                   const CascIO& io, const float* sc, hipStream_t st)
{
    march::FieldOpIncl<kInclSlots> op{};
    op.Fb = Fb;
    op.fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    for (int w = 0; w < kInclSlots; ++w) op.sc[w] = sc[w];
    return launch_fs_up(L, nx, nz, op, march::StoreEpiSlots<kInclSlots>{(float*)io.out, io.slot_stride}, dirs, io, st);
}

hipError_t launch_march_fix_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb, const double4* dirs,
                                 const CascIO& io, const float* sc, hipStream_t st)
{
    march::FieldOpIncl<kInclSlots> op{};
    op.Fb = Fb;
    op.fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    for (int w = 0; w < kInclSlots; ++w) op.sc[w] = sc[w];
    march::UpF32 up{(const float*)io.up};
    up.stride = io.slot_stride;
    return launch_fix_k(L, nx, nz, op, march::StoreEpiSlots<kInclSlots>{(float*)io.out, io.slot_stride}, dirs, up, st);
}

hipError_t launch_march_merge_j_incl(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb,
                                     const double4* dirs, const CascIO& io, float* J, int32_t lam0, int32_t n_valid,
                                     const float* sc, const float* wt, hipStream_t st)
{
    march::FieldOpIncl<kInclSlots> op{};
    op.Fb = Fb;
    op.fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    march::JEpiIncl<kInclSlots> epi{J, lam0, n_valid, (int64_t)nx * nz, {}};
    for (int w = 0; w < kInclSlots; ++w) {
        op.sc[w] = sc[w];
        epi.wt[w] = wt[w];
    }
    return launch_fs_up(L, nx, nz, op, epi, dirs, io, st);
}

hipError_t launch_mask_fields(float2* F, const uint8_t* mask, int64_t ncell, int32_t n_batch, hipStream_t st)
{
    const int64_t n = (int64_t)n_batch * ncell * kLB;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_mask_fields, dim3(blocks), dim3(256), 0, st, F, mask, ncell, n_batch);
    return hipGetLastError();
}

hipError_t launch_mask_j(float* J, const uint8_t* mask, int64_t ncell, int32_t n_wave, hipStream_t st)
{
    const int64_t n = (int64_t)n_wave * ncell;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_mask_j, dim3(blocks), dim3(256), 0, st, J, mask, ncell, n_wave);
    return hipGetLastError();
}

hipError_t launch_j(const float* I0, float* J, int32_t lam0, int32_t n_valid, int64_t ncell, int32_t n0, float w,
                    bool acc, hipStream_t st)
{
    dim3 grid((unsigned)((ncell + 63) / 64));
    hipLaunchKernelGGL(k_j, grid, dim3(256), 0, st, I0, J, lam0, n_valid, ncell, n0, w, (int32_t)acc);
    return hipGetLastError();
}

}  // namespace rcx
