// fs_kernels.hip -- gfx950 kernels of the radiance-cascades formal solution
// (Osborne & Sannikov, arXiv:2408.14425, Secs. 2.2-2.3 and 3.2).
//
// Data layout in HBM (x fastest within a cell index c = z * nx + x):
//   F      [c][lambda]            float2 {chi * voxel (floored at 1e-20), S = eta/chi}
//   cascade[(p * N_i + k)][lambda] float  merged radiance of probe p, direction k
//   J      [lambda][c]            float  (the caller's layout)
// Wavelength is the fastest index of F and of the cascades: a wavefront of 64
// lanes holds 64 wavelengths of one ray, so the cell walk is wave-uniform and
// every step reads 64 contiguous {chi, S} pairs.
#include "rcx_internal.h"

#include <cmath>

namespace rcx {

namespace {

constexpr int kBlock = 256;
constexpr unsigned kXcds = 8;

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of logical blocks so rays that share cells share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    unsigned per = nb / kXcds, rem = nb % kXcds;
    unsigned x = b % kXcds, slot = b / kXcds;
    unsigned start = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return start + slot;
}

// 1 - e^{-x} for x >= 0 without cancellation: a short series below 1/8,
// the direct form above (where its relative error is below 1e-6).
__device__ __forceinline__ float one_minus_exp_neg(float x, float e)
{
    float ser = x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f)))));
    return x < 0.125f ? ser : 1.0f - e;
}

// ---------------------------------------------------------------- prep
// chi, eta [n_wave][ncell] -> F [ncell][n_wave] through a 32x32 LDS tile.
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ chi,
                                              const float* __restrict__ eta,
                                              float2* __restrict__ F, int32_t n_wave,
                                              int64_t ncell, float voxel)
{
    __shared__ float2 tile[32][33];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * 32;
    const int32_t l0 = blockIdx.y * 32;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int32_t l = l0 + ty + 8 * r;
        int64_t c = c0 + tx;
        float2 v = make_float2(0.0f, 0.0f);
        if (l < n_wave && c < ncell) {
            float ch = chi[(int64_t)l * ncell + c];
            float et = eta[(int64_t)l * ncell + c];
            float cv = ch * voxel;
            const float floor_c = 1e-20f;
            if (cv >= floor_c) {
                v = make_float2(cv, et / ch);
            } else {
                v = make_float2(floor_c, et * voxel / floor_c);
            }
        }
        tile[ty + 8 * r][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int64_t c = c0 + ty + 8 * r;
        int32_t l = l0 + tx;
        if (l < n_wave && c < ncell) F[c * n_wave + l] = tile[tx][ty + 8 * r];
    }
}

// ------------------------------------------------------- march + merge
// One lane per (ray, wavelength), wavelength fastest. The ray of cascade i
// from probe (u, v) along direction k covers [ta, tb) clipped to the domain.
// Cells are walked front to back with the plane crossings computed in FP64
// (exact cell boundaries; the radiative arithmetic is FP32):
//   I += T S (1 - e^{-dtau}),  T *= e^{-dtau}
// which equals the back-to-front piecewise-constant solution of Sec. 3.2.
// The merge with the cascade above (Sec. 2.3.1) follows in the same lane:
//   Itilde = I + T * sum_taps w_x w_z (1/4) sum_j Itilde_up(tap, 4k + j).
__global__ __launch_bounds__(kBlock) void k_march_merge(LevelDesc L, int32_t nx, int32_t nz,
                                                         int32_t n_wave, const float2* __restrict__ F,
                                                         const double4* __restrict__ dirs,
                                                         const float* __restrict__ up,
                                                         float* __restrict__ out, int64_t total)
{
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t idx = (int64_t)lb * kBlock + threadIdx.x; idx < total; idx += stride) {
        const int64_t ray = idx / n_wave;
        const int32_t lam = (int32_t)(idx - ray * n_wave);
        const int32_t k = (int32_t)(ray % L.nd);
        const int32_t p = (int32_t)(ray / L.nd);
        const int32_t u = p % L.px, v = p / L.px;

        const double cx = (u + 0.5) * L.s, cz = (v + 0.5) * L.s;
        const double4 d = dirs[k];  // {wx, wz, 1/wx, 1/wz}
        // slab clip to [0, nx] x [0, nz]
        double ax = (0.0 - cx) * d.z, bx = ((double)nx - cx) * d.z;
        double az = (0.0 - cz) * d.w, bz = ((double)nz - cz) * d.w;
        double lo = fmax(L.ta, fmax(fmin(ax, bx), fmin(az, bz)));
        double hi = fmin(L.tb, fmin(fmax(ax, bx), fmax(az, bz)));

        float I = 0.0f, T = 1.0f;
        if (lo < hi) {
            const int sx = d.x > 0.0 ? 1 : -1;
            const int sz = d.y > 0.0 ? 1 : -1;
            double x0 = cx + lo * d.x, z0 = cz + lo * d.y;
            int ix = d.x > 0.0 ? (int)floor(x0) : (int)ceil(x0) - 1;
            int iz = d.y > 0.0 ? (int)floor(z0) : (int)ceil(z0) - 1;
            ix = min(max(ix, 0), nx - 1);
            iz = min(max(iz, 0), nz - 1);
            // the next x (z) plane the ray crosses, as an integer coordinate
            int Xn = d.x > 0.0 ? ix + 1 : ix;
            int Zn = d.y > 0.0 ? iz + 1 : iz;
            double tnx = ((double)Xn - cx) * d.z;
            double tnz = ((double)Zn - cz) * d.w;
            double t = lo;
            for (int step = 0; step < L.max_steps; ++step) {
                const bool xs = tnx <= tnz;
                const double te = fmin(xs ? tnx : tnz, hi);
                const float ds = (float)(te - t);
                const int cxi = min(max(ix, 0), nx - 1);
                const int czi = min(max(iz, 0), nz - 1);
                const float2 f = F[((int64_t)czi * nx + cxi) * n_wave + lam];
                const float dtau = f.x * ds;
                const float e = __expf(-dtau);
                I = fmaf(T * f.y, one_minus_exp_neg(dtau, e), I);
                T *= e;
                t = te;
                if (te >= hi) break;
                if (xs) {
                    ix += sx;
                    Xn += sx;
                    tnx = ((double)Xn - cx) * d.z;
                } else {
                    iz += sz;
                    Zn += sz;
                    tnz = ((double)Zn - cz) * d.w;
                }
            }
        }

        if (L.has_up) {
            // Bilinear taps on the cascade above: q = (u + 1/2)/2 - 1/2, so
            // even u -> taps (u/2 - 1, u/2) with weights (1/4, 3/4), odd u ->
            // taps ((u-1)/2, (u+1)/2) with weights (3/4, 1/4); clamped.
            const int bx0 = (u - 1) >> 1, bz0 = (v - 1) >> 1;
            const float fx = (u & 1) ? 0.25f : 0.75f;
            const float fz = (v & 1) ? 0.25f : 0.75f;
            const int tx0 = min(max(bx0, 0), L.qx - 1), tx1 = min(max(bx0 + 1, 0), L.qx - 1);
            const int tz0 = min(max(bz0, 0), L.qz - 1), tz1 = min(max(bz0 + 1, 0), L.qz - 1);
            const int txs[2] = {tx0, tx1};
            const int tzs[2] = {tz0, tz1};
            const float wxs[2] = {1.0f - fx, fx};
            const float wzs[2] = {1.0f - fz, fz};
            float far = 0.0f;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int64_t base =
                        (((int64_t)tzs[a] * L.qx + txs[b]) * L.nd_up + 4 * (int64_t)k) * n_wave + lam;
                    float c = up[base] + up[base + n_wave] + up[base + 2 * n_wave] + up[base + 3 * n_wave];
                    far = fmaf(wzs[a] * wxs[b], 0.25f * c, far);
                }
            I = fmaf(T, far, I);
        }
        out[ray * n_wave + lam] = I;
    }
}

// ---------------------------------------------------------------- J
// J[lambda][c] = (1/N_0) sum_k Itilde_0[(c * N_0 + k)][lambda], transposed
// through a 32x32 LDS tile.
__global__ __launch_bounds__(256) void k_j(const float* __restrict__ I0, float* __restrict__ J,
                                           int32_t n_wave, int64_t ncell, int32_t n0)
{
    __shared__ float tile[32][33];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * 32;
    const int32_t l0 = blockIdx.y * 32;
    const float inv = 1.0f / (float)n0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int64_t c = c0 + ty + 8 * r;
        int32_t l = l0 + tx;
        float acc = 0.0f;
        if (l < n_wave && c < ncell) {
            for (int k = 0; k < n0; ++k) acc += I0[(c * n0 + k) * n_wave + l];
        }
        tile[ty + 8 * r][tx] = acc * inv;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int32_t l = l0 + ty + 8 * r;
        int64_t c = c0 + tx;
        if (l < n_wave && c < ncell) J[(int64_t)l * ncell + c] = tile[tx][ty + 8 * r];
    }
}

}  // namespace

hipError_t launch_prep(const float* chi, const float* eta, float2* F, int32_t n_wave, int64_t ncell,
                       float voxel, hipStream_t st)
{
    dim3 grid((unsigned)((ncell + 31) / 32), (unsigned)((n_wave + 31) / 32));
    hipLaunchKernelGGL(k_prep, grid, dim3(32, 8), 0, st, chi, eta, F, n_wave, ncell, voxel);
    return hipGetLastError();
}

hipError_t launch_march_merge(const LevelDesc& L, int32_t nx, int32_t nz, int32_t n_wave,
                              const float2* F, const double4* dirs, const float* up, float* out,
                              hipStream_t st)
{
    const int64_t total = (int64_t)L.px * L.pz * L.nd * n_wave;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    const int64_t cap = 1 << 22;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_march_merge, dim3((unsigned)blocks), dim3(kBlock), 0, st, L, nx, nz, n_wave,
                       F, dirs, up, out, total);
    return hipGetLastError();
}

hipError_t launch_j(const float* I0, float* J, int32_t n_wave, int64_t ncell, int32_t n0,
                    hipStream_t st)
{
    dim3 grid((unsigned)((ncell + 31) / 32), (unsigned)((n_wave + 31) / 32));
    hipLaunchKernelGGL(k_j, grid, dim3(32, 8), 0, st, I0, J, n_wave, ncell, n0);
    return hipGetLastError();
}

}  // namespace rcx
