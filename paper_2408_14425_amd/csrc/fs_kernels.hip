// fs_kernels.hip -- gfx950 kernels of the radiance-cascades formal solution
// (Osborne & Sannikov, arXiv:2408.14425, Secs. 2.2-2.3 and 3.2).
//
// Wavelengths are processed in batches of 16 (kLB). Data layout in HBM, with
// c = z * nx + x the cell index and l the wavelength within a batch:
//   F       [batch][c][16]          float2 {chi * voxel * log2(e) (floored), S = eta/chi}
//   cascade [(p * N_i + k)][16]     float  merged radiance of probe p, direction k
//   J       [lambda][c]             float  (the caller's layout)
// A batch of F is 128 MB at 1024^2, so it stays resident in the 256 MB
// Infinity Cache while every cascade of that batch is marched.
//
// A wavefront holds 4 rays x 16 wavelengths: each 16-lane row is one ray.
// The cell walk is done cooperatively per row: lane j computes the one or
// two segments of the j-th grid column the ray crosses along its major axis
// (plane crossings in FP64, so cell boundaries are exact), the row compacts
// them into LDS, and all 16 wavelength lanes then step through the list with
// the FP32 radiative update.
#include "rcx_internal.h"

#include <cmath>

namespace rcx {

namespace {

constexpr int kBlock = 256;                    // 4 wavefronts
constexpr int kRaysPerBlock = (kBlock / 64) * 4;  // 4 rows of 16 lanes per wavefront
constexpr int kLB = 16;      // wavelengths per batch = lanes per row
constexpr unsigned kXcds = 8;
constexpr float kChiFloor = 1e-20f;     // per cell, natural units
constexpr float kLog2e = 1.4426950408889634f;
constexpr uint32_t kOob = 0x80000000u;  // buffer offset past every field slice: loads return 0

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of logical blocks so rays that share cells share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    unsigned per = nb / kXcds, rem = nb % kXcds;
    unsigned x = b % kXcds, slot = b / kXcds;
    unsigned start = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return start + slot;
}

// 1 - 2^{-y} for y >= 0 (y = optical depth in log2 units) without
// cancellation: with x = y ln2, the series x - x^2/2 + x^3/6 below x = 1/64
// (truncation < 2e-7 relative), the direct form above (< 4e-6 relative).
__device__ __forceinline__ float one_minus_exp2_neg(float y, float e)
{
    constexpr float c1 = 0.6931471805599453f;   // ln 2
    constexpr float c2 = 0.2402265069591007f;   // (ln 2)^2 / 2
    constexpr float c3 = 0.0555041086648216f;   // (ln 2)^3 / 6
    const float ser = y * (c1 - y * (c2 - y * c3));
    return y < (1.0f / 64.0f) / c1 ? ser : 1.0f - e;
}

// ---------------------------------------------------------------- prep
// chi, eta [n_wave][ncell] -> F [batch][ncell][16], one 64-cell x 16-wavelength
// tile per block through LDS. Wavelengths past n_wave are padded with
// {1, 0} (no emission).
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ chi,
                                              const float* __restrict__ eta,
                                              float2* __restrict__ F, int32_t n_wave,
                                              int64_t ncell, float voxel)
{
    __shared__ float2 tile[kLB][65];
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
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = t & 15;
        const int cc = (t >> 4) + 16 * r;
        const int64_t c = c0 + cc;
        if (c < ncell) F[((int64_t)b * ncell + c) * kLB + l] = tile[l][cc];
    }
}

// ------------------------------------------------------- march + merge
// Ray `ray` of cascade i (probe p = ray / N_i, direction k = ray % N_i)
// covers [ta, tb) clipped to the domain. Front-to-back accumulation
//   I += T S (1 - e^{-dtau}),  T *= e^{-dtau}
// equals the back-to-front piecewise-constant solution of Sec. 3.2. The
// merge with the cascade above (Sec. 2.3.1) follows:
//   Itilde = I + T * sum_taps w_x w_z (1/4) sum_j Itilde_up(tap, 4k + j).
__global__ __launch_bounds__(kBlock) void k_march_rows(LevelDesc L, int32_t nx, int32_t nz,
                                                        const float2* __restrict__ Fb, uint32_t fb_bytes,
                                                        const double4* __restrict__ dirs,
                                                        const float* __restrict__ up,
                                                        float* __restrict__ out, int64_t total)
{
    // per wave, per row: (byte offset of the cell's wavelength row in F, ds) entries
    __shared__ uint4 seg[kBlock / 64][4][16];

    const __amdgpu_buffer_rsrc_t frsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)Fb, 0, (int)fb_bytes, 0x00020000);

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int row = lane >> 4;
    const int l = lane & 15;
    const uint64_t row_bits = 0xFFFFull << (16 * row);
    const uint64_t lt_bits = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t lane_off = (uint32_t)l * 8u;
    // Entries never written in a chunk must read as "no cell, no length".
    {
        uint4* sw = &seg[w][0][0];
        sw[lane] = make_uint4(kOob, 0u, kOob, 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * kRaysPerBlock;
    for (int64_t base = ((int64_t)lb * (kBlock / 64) + w) * 4; base < total; base += stride) {
        const int64_t ray = base + row;
        const bool active = ray < total;
        const int64_t rr = active ? ray : total - 1;
        const int32_t k = (int32_t)(rr % L.nd);
        const int32_t p = (int32_t)(rr / L.nd);
        const int32_t u = p % L.px, v = p / L.px;

        const double cx = (u + 0.5) * L.s, cz = (v + 0.5) * L.s;
        const double4 d = dirs[k];  // {wx, wz, 1/wx, 1/wz}
        // Plane crossings t(X) = X / w - c / w, evaluated with one FMA so the
        // crossing of the domain's exit plane equals the clip bound exactly.
        const double offx = -cx * d.z, offz = -cz * d.w;
        const double ax = offx, bx = fma((double)nx, d.z, offx);
        const double az = offz, bz = fma((double)nz, d.w, offz);
        double lo = fmax(L.ta, fmax(fmin(ax, bx), fmin(az, bz)));
        double hi = fmin(L.tb, fmin(fmax(ax, bx), fmax(az, bz)));
        if (!active) {
            lo = 1.0;
            hi = 0.0;
        }

        // Major axis m (the one crossed at least as often), minor axis n.
        const bool xmaj = fabs(d.x) >= fabs(d.y);
        const double wm = xmaj ? d.x : d.y, wn = xmaj ? d.y : d.x;
        const double cm = xmaj ? cx : cz, cn = xmaj ? cz : cx;
        const double im_ = xmaj ? d.z : d.w, in_ = xmaj ? d.w : d.z;
        const double offm = xmaj ? offx : offz, offn = xmaj ? offz : offx;
        const int nm = xmaj ? nx : nz, nn = xmaj ? nz : nx;
        const int strm = xmaj ? 1 : nx, strn = xmaj ? nx : 1;
        const int sm = wm > 0.0 ? 1 : -1, sn = wn > 0.0 ? 1 : -1;

        const double pm0 = cm + lo * wm;
        int im0 = wm > 0.0 ? (int)floor(pm0) : (int)ceil(pm0) - 1;
        im0 = min(max(im0, 0), nm - 1);
        const int mfirst = wm > 0.0 ? im0 + 1 : im0;  // first m-plane crossed

        float I = 0.0f, T = 1.0f;
        const int max_chunks = (nm + 2 + 15) / 16 + 1;
        for (int chunk = 0; chunk < max_chunks; ++chunk) {
            // ---- column j of this row's ray: one or two segments
            const int j = chunk * 16 + l;
            const double ta = (j == 0) ? lo : fma((double)(mfirst + (j - 1) * sm), im_, offm);
            const double tb_ = fmin(fma((double)(mfirst + j * sm), im_, offm), hi);
            const bool valid = ta < hi;
            const int im = min(max(im0 + j * sm, 0), nm - 1);
            const double pn = cn + ta * wn;
            int in0 = wn > 0.0 ? (int)floor(pn) : (int)ceil(pn) - 1;
            in0 = min(max(in0, 0), nn - 1);
            const int nnext = wn > 0.0 ? in0 + 1 : in0;
            const double tn = fma((double)nnext, in_, offn);
            const bool two = valid && tn < tb_;
            const double tmid = fmax(tn, ta);
            const uint32_t cell1 = (uint32_t)(im * strm + in0 * strn) * (uint32_t)(kLB * 8);
            const int in1 = min(max(in0 + sn, 0), nn - 1);
            const uint32_t cell2 = (uint32_t)(im * strm + in1 * strn) * (uint32_t)(kLB * 8);
            const float ds1 = (float)fmax((two ? tmid : tb_) - ta, 0.0);
            const float ds2 = (float)fmax(tb_ - tmid, 0.0);

            const uint64_t b1 = __ballot(valid);
            if (b1 == 0) break;
            const uint64_t b2 = __ballot(two);
            const int pos = __popcll(b1 & row_bits & lt_bits) + __popcll(b2 & row_bits & lt_bits);
            const int n_row = __popcll(b1 & row_bits) + __popcll(b2 & row_bits);
            int n_max = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t rb = 0xFFFFull << (16 * q);
                n_max = max(n_max, __popcll(b1 & rb) + __popcll(b2 & rb));
            }
            uint2* srow = reinterpret_cast<uint2*>(&seg[w][row][0]);
            if (valid) srow[pos] = make_uint2(cell1, __float_as_uint(ds1));
            if (two) srow[pos + 1] = make_uint2(cell2, __float_as_uint(ds2));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            // ---- step through the row's segments, 4 at a time. Positions past
            // the row's count load from an out-of-range offset (value 0: no
            // opacity, no emission) and leave I and T unchanged.
            // ---- step through the row's segments, 4 at a time. Positions past
            // the row's count load from an out-of-range offset (value 0: no
            // opacity, no emission) and leave I and T unchanged.
            for (int s = 0; s < n_max; s += 4) {
                const uint4 e01 = seg[w][row][s >> 1];
                const uint4 e23 = seg[w][row][(s >> 1) + 1];
                const uint32_t offs[4] = {e01.x, e01.z, e23.x, e23.z};
                const float dsv[4] = {__uint_as_float(e01.y), __uint_as_float(e01.w), __uint_as_float(e23.y),
                                      __uint_as_float(e23.w)};
                float2 f[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t off = (s + q < n_row) ? offs[q] + lane_off : kOob;
                    f[q] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(frsrc, off, 0, 0));
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float y = f[q].x * dsv[q];  // optical depth, log2 units
                    const float e = __builtin_amdgcn_exp2f(-y);
                    I = fmaf(T * f[q].y, one_minus_exp2_neg(y, e), I);
                    T *= e;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }

        if (active) {
            if (L.has_up) {
                // Bilinear taps on the cascade above: q = (u + 1/2)/2 - 1/2, so
                // even u -> taps (u/2 - 1, u/2) with weights (1/4, 3/4), odd u ->
                // taps ((u-1)/2, (u+1)/2) with weights (3/4, 1/4); clamped.
                const int bx0 = (u - 1) >> 1, bz0 = (v - 1) >> 1;
                const float fx = (u & 1) ? 0.25f : 0.75f;
                const float fz = (v & 1) ? 0.25f : 0.75f;
                const int txs[2] = {min(max(bx0, 0), L.qx - 1), min(max(bx0 + 1, 0), L.qx - 1)};
                const int tzs[2] = {min(max(bz0, 0), L.qz - 1), min(max(bz0 + 1, 0), L.qz - 1)};
                const float wxs[2] = {1.0f - fx, fx};
                const float wzs[2] = {1.0f - fz, fz};
                float far = 0.0f;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) {
                        const int64_t bi =
                            (((int64_t)tzs[a] * L.qx + txs[bb]) * L.nd_up + 4 * (int64_t)k) * kLB + l;
                        const float c4 = up[bi] + up[bi + kLB] + up[bi + 2 * kLB] + up[bi + 3 * kLB];
                        far = fmaf(wzs[a] * wxs[bb], 0.25f * c4, far);
                    }
                I = fmaf(T, far, I);
            }
            out[ray * kLB + l] = I;
        }
    }
}

// ---------------------------------------------------------------- J
// J[16 b + l][c] = (1/N_0) sum_k Itilde_0[(c * N_0 + k)][l] for one batch,
// through a 64-cell x 16-wavelength LDS tile.
__global__ __launch_bounds__(256) void k_j(const float* __restrict__ I0, float* __restrict__ J,
                                           int32_t n_wave, int32_t batch, int64_t ncell, int32_t n0)
{
    __shared__ float tile[kLB][65];
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const float inv = 1.0f / (float)n0;
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
        const int32_t lam = batch * kLB + l;
        const int64_t c = c0 + cc;
        if (lam < n_wave && c < ncell) J[(int64_t)lam * ncell + c] = tile[l][cc];
    }
}

}  // namespace

int32_t batch_width() { return kLB; }

hipError_t launch_prep(const float* chi, const float* eta, float2* F, int32_t n_wave, int64_t ncell,
                       float voxel, hipStream_t st)
{
    dim3 grid((unsigned)((ncell + 63) / 64), (unsigned)((n_wave + kLB - 1) / kLB));
    hipLaunchKernelGGL(k_prep, grid, dim3(256), 0, st, chi, eta, F, n_wave, ncell, voxel);
    return hipGetLastError();
}

hipError_t launch_march_merge(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb,
                              const double4* dirs, const float* up, float* out, hipStream_t st)
{
    const uint32_t fb_bytes = (uint32_t)((int64_t)nx * nz * kLB * sizeof(float2));
    const int64_t total = (int64_t)L.px * L.pz * L.nd;  // rays
    int64_t blocks = (total + kRaysPerBlock - 1) / kRaysPerBlock;
    const int64_t cap = 1 << 20;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_march_rows, dim3((unsigned)blocks), dim3(kBlock), 0, st, L, nx, nz, Fb, fb_bytes,
                       dirs, up, out, total);
    return hipGetLastError();
}

hipError_t launch_j(const float* I0, float* J, int32_t n_wave, int32_t batch, int64_t ncell, int32_t n0,
                    hipStream_t st)
{
    dim3 grid((unsigned)((ncell + 63) / 64));
    hipLaunchKernelGGL(k_j, grid, dim3(256), 0, st, I0, J, n_wave, batch, ncell, n0);
    return hipGetLastError();
}

}  // namespace rcx
