// mlp.hip -- the warm-start multilayer perceptron on gfx950: BF16 MFMA
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation, FP32 master weights,
// Adam. Network: x [B][n_in] -> (Linear, SiLU) x depth -> Linear -> y [B][n_out].
//
// Every product is one "NT" GEMM, C[m][n] = sum_k A[m][k] B[n][k], with both
// operands stored k-contiguous (bf16):
//   forward        Z_l  = H_{l-1} W_l        A = H_{l-1} [B][K],  B = W_l^T [N][K]
//   backward data  dH   = dZ_l W_l^T         A = dZ_l [B][N],     B = W_l [K][N]
//   weight grad    dW_l = H_{l-1}^T dZ_l     A = H^T [K][B],      B = dZ^T [N][B]
// so the epilogues also write the transposed copies H^T and dZ^T the weight
// gradient needs. A workgroup of 4 wavefronts computes a 64 x 64 tile, each
// wavefront one 32 x 32 MFMA block; the weight gradient splits the batch
// (its contraction) over workgroups and reduces the partial tiles in a fixed
// order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rcx_internal.h"

namespace rcx {
namespace mlpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 64;
constexpr int kKStep = 16;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

enum Epi : int { kFwdHidden = 0, kFwdOut = 1, kBwdData = 2, kWGrad = 3 };

struct GemmArgs {
    const __bf16* A;  // [M][lda]
    const __bf16* B;  // [N][ldb]
    int32_t M, N, K, lda, ldb;
    int32_t k_split;  // weight gradient: K range per split
    // epilogue
    const float* bias;   // [N] (forward)
    float* Z;            // forward hidden: pre-activation [M][N]; backward: reads Z of the layer below
    __bf16* H;           // forward hidden: activation [M][ldh]; backward: dZ [M][ldh]
    __bf16* Ht;          // transposed copy [N][ldt]
    int32_t ldh, ldt, ldz;
    float* Y;            // forward output [M][n_valid]
    int32_t n_valid;     // columns that exist (padding beyond is dropped / zeroed)
    float* P;            // weight-gradient partials [split][M][N]
};

// MFMA 32x32x16 operand layout (wave64): lane l holds row (l % 32) and the 8
// consecutive k values starting at 8 (l / 32); the accumulator's register r
// holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int m0 = blockIdx.x * kTile + (w >> 1) * 32;
    const int n0 = blockIdx.y * kTile + (w & 1) * 32;
    const int kbeg = (EPI == kWGrad) ? blockIdx.z * g.k_split : 0;
    const int kend = (EPI == kWGrad) ? min(g.K, kbeg + g.k_split) : g.K;
    const int r = lane & 31, kg = (lane >> 5) * 8;
    const int am = m0 + r, bn = n0 + r;
    f32x16 acc = {};
    for (int k = kbeg; k < kend; k += kKStep) {
        bf16x8 a = {}, b = {};
        if (am < g.M) a = *reinterpret_cast<const bf16x8*>(g.A + (int64_t)am * g.lda + k + kg);
        if (bn < g.N) b = *reinterpret_cast<const bf16x8*>(g.B + (int64_t)bn * g.ldb + k + kg);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const int col = n0 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = m0 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (row >= g.M || col >= g.N) continue;
        const float v = acc[q];
        if (EPI == kFwdHidden) {
            const float z = v + g.bias[col];
            const float h = silu(z);
            g.Z[(int64_t)row * g.ldz + col] = z;
            g.H[(int64_t)row * g.ldh + col] = (__bf16)h;
            g.Ht[(int64_t)col * g.ldt + row] = (__bf16)h;
        } else if (EPI == kFwdOut) {
            if (col < g.n_valid) g.Y[(int64_t)row * g.n_valid + col] = v + g.bias[col];
        } else if (EPI == kBwdData) {
            const float dz = v * dsilu(g.Z[(int64_t)row * g.ldz + col]);
            g.H[(int64_t)row * g.ldh + col] = (__bf16)dz;
            g.Ht[(int64_t)col * g.ldt + row] = (__bf16)dz;
        } else {
            g.P[((int64_t)blockIdx.z * g.M + row) * g.N + col] = v;
        }
    }
}

// x [B][n_in] fp32 -> A0 [Bp][16] bf16 (zero padded) and A0^T [16][Bp].
__global__ void k_pack_input(const float* __restrict__ x, int32_t B, int32_t Bp, int32_t n_in, __bf16* __restrict__ A0,
                             __bf16* __restrict__ A0t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Bp * 16) return;
    const int64_t b = i / 16;
    const int c = (int)(i % 16);
    const float v = (b < B && c < n_in) ? x[b * n_in + c] : 0.0f;
    A0[i] = (__bf16)v;
    A0t[(int64_t)c * Bp + b] = (__bf16)v;
}

// Loss gradient dL/dy = 2 (y - y_ref) / (B n_out) -> dZ [Bp][ld] and dZ^T, and
// per-block partial sums of the squared error.
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ yref, int32_t B, int32_t Bp,
                            int32_t n_out, int32_t ld, __bf16* __restrict__ dZ, __bf16* __restrict__ dZt,
                            float* __restrict__ loss_part)
{
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float se = 0.0f;
    if (i < (int64_t)Bp * ld) {
        const int64_t b = i / ld;
        const int c = (int)(i % ld);
        float d = 0.0f;
        if (b < B && c < n_out) {
            const float e = y[b * n_out + c] - yref[b * n_out + c];
            se = e * e;
            d = 2.0f * e / ((float)B * (float)n_out);
        }
        dZ[i] = (__bf16)d;
        dZt[(int64_t)c * Bp + b] = (__bf16)d;
    }
    red[threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Weight gradient: sum the split partials (fixed order); bias gradient: row
// sums of dZ^T (one wavefront per output column, fixed order).
__global__ void k_wgrad_reduce(const float* __restrict__ P, int32_t splits, int32_t K, int32_t N, int32_t k_valid,
                               int32_t n_valid, float* __restrict__ gW)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)k_valid * n_valid) return;
    const int k = (int)(i / n_valid), n = (int)(i % n_valid);
    float s = 0.0f;
    for (int p = 0; p < splits; ++p) s += P[((int64_t)p * K + k) * N + n];
    gW[i] = s;
}

// Bias gradient: gb[n] = sum over the batch of dZ^T[n][.]. One block of 256
// threads per output; each thread sums 8 consecutive values per 16-byte load
// (rows are 128-byte aligned: Bp is a multiple of 64), the block reduces in
// a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_bias_grad(const __bf16* __restrict__ dZt, int32_t Bp, int32_t n_valid,
                                                   float* __restrict__ gb)
{
    __shared__ float part[4];
    const int n = blockIdx.x;
    if (n >= n_valid) return;
    const uint4* row = reinterpret_cast<const uint4*>(dZt + (int64_t)n * Bp);
    const int n8 = Bp / 8;
    float s = 0.0f;
    for (int i = threadIdx.x; i < n8; i += 256) {
        const uint4 q = row[i];
        const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            s += __uint_as_float(wv[h] << 16);
            s += __uint_as_float(wv[h] & 0xFFFF0000u);
        }
    }
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gb[n] = (part[0] + part[1]) + (part[2] + part[3]);
}

// Adam on the flat FP32 parameters, then refresh the bf16 copies W [Kp][Np]
// (k-major, for backward data) and W^T [Np][Kp] (for forward) of one layer.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_layer_copies(const float* __restrict__ W, const float* __restrict__ b, int32_t fan_in, int32_t fan_out,
                               int32_t Kp, int32_t Np, __bf16* __restrict__ Wk, __bf16* __restrict__ Wt,
                               float* __restrict__ bias_p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)Kp * Np) {
        const int k = (int)(i / Np), nn = (int)(i % Np);
        const float w = (k < fan_in && nn < fan_out) ? W[(int64_t)k * fan_out + nn] : 0.0f;
        Wk[(int64_t)k * Np + nn] = (__bf16)w;
        Wt[(int64_t)nn * Kp + k] = (__bf16)w;
    }
    if (i < Np) bias_p[i] = (i < fan_out) ? b[i] : 0.0f;
}

}  // namespace mlpk
}  // namespace rcx

// ====================================================================== host

using namespace rcx;
using namespace rcx::mlpk;

struct rcx_mlp {
    int32_t n_in, width, depth, n_out, max_batch, Bp_max;
    int32_t n_layers;
    std::vector<int32_t> fin, fout, Kp, Np;  // per layer: true and padded fan-in / fan-out
    std::vector<int64_t> off;                // offset of layer l's W in the flat parameters (b follows)
    int64_t n_params = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // flat FP32
    std::vector<__bf16*> Wk, Wt;
    std::vector<float*> bias;
    std::vector<__bf16*> Hs, Hts;  // activations per layer input: [Bp][Kp], [Kp][Bp]
    std::vector<float*> Zs;        // pre-activations of hidden layers [Bp][Np]
    __bf16 *dA = nullptr, *dAt = nullptr, *dB = nullptr, *dBt = nullptr;  // backward ping-pong [Bp][128]
    float* Y = nullptr;
    float* P = nullptr;  // weight-gradient partials
    float* loss_part = nullptr;
    int64_t t = 0;
    std::vector<void*> allocs;
};

namespace {

constexpr int kSplits = 64;

int32_t rup(int32_t x, int32_t m) { return (x + m - 1) / m * m; }

template <class P>
hipError_t dalloc(rcx_mlp* s, P** p, size_t bytes)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) {
        s->allocs.push_back(q);
        (void)hipMemset(q, 0, std::max<size_t>(bytes, 256));
    }
    *p = (P*)q;
    return e;
}

unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t refresh_copies(rcx_mlp* s, hipStream_t st)
{
    for (int l = 0; l < s->n_layers; ++l) {
        const float* W = s->p + s->off[l];
        const float* b = W + (int64_t)s->fin[l] * s->fout[l];
        const int64_t n = (int64_t)s->Kp[l] * s->Np[l];
        hipLaunchKernelGGL(k_layer_copies, dim3(nblk(n, 256)), dim3(256), 0, st, W, b, s->fin[l], s->fout[l], s->Kp[l],
                           s->Np[l], s->Wk[l], s->Wt[l], s->bias[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int EPI>
hipError_t gemm(const GemmArgs& g, int splits, hipStream_t st)
{
    dim3 grid(nblk(g.M, kTile), nblk(g.N, kTile), splits);
    hipLaunchKernelGGL(k_gemm_nt<EPI>, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t forward(rcx_mlp* s, const float* x, float* y, int32_t B, int32_t Bp, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_input, dim3(nblk((int64_t)Bp * 16, 256)), dim3(256), 0, st, x, B, Bp, s->n_in, s->Hs[0],
                       s->Hts[0]);
    hipError_t e = hipGetLastError();
    for (int l = 0; l < s->n_layers && e == hipSuccess; ++l) {
        GemmArgs g{};
        g.A = s->Hs[l];
        g.lda = s->Kp[l];
        g.B = s->Wt[l];
        g.ldb = s->Kp[l];
        g.M = Bp;
        g.N = s->Np[l];
        g.K = s->Kp[l];
        g.bias = s->bias[l];
        if (l < s->n_layers - 1) {
            g.Z = s->Zs[l];
            g.ldz = s->Np[l];
            g.H = s->Hs[l + 1];
            g.ldh = s->Np[l];
            g.Ht = s->Hts[l + 1];
            g.ldt = Bp;
            e = gemm<kFwdHidden>(g, 1, st);
        } else {
            g.Y = y;
            g.n_valid = s->fout[l];
            g.M = B;
            e = gemm<kFwdOut>(g, 1, st);
        }
    }
    return e;
}

// Gradients of the MSE loss into s->g (flat, FP32). Returns the loss sum
// partials in s->loss_part (nblk blocks).
hipError_t backward(rcx_mlp* s, const float* yref, int32_t B, int32_t Bp, int* n_loss_blocks, hipStream_t st)
{
    const int L = s->n_layers;
    const int ld_out = s->Np[L - 1];
    const int64_t nl = (int64_t)Bp * ld_out;
    *n_loss_blocks = (int)nblk(nl, 256);
    hipLaunchKernelGGL(k_loss_grad, dim3(*n_loss_blocks), dim3(256), 0, st, s->Y, yref, B, Bp, s->n_out, ld_out, s->dA,
                       s->dAt, s->loss_part);
    hipError_t e = hipGetLastError();
    __bf16 *dZ = s->dA, *dZt = s->dAt, *dN = s->dB, *dNt = s->dBt;
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        // weight gradient dW_l [Kp][Np] = H_l^T dZ_l, split over the batch
        GemmArgs gw{};
        gw.A = s->Hts[l];
        gw.lda = Bp;
        gw.B = dZt;
        gw.ldb = Bp;
        gw.M = s->Kp[l];
        gw.N = s->Np[l];
        gw.K = Bp;
        gw.k_split = rup((Bp + kSplits - 1) / kSplits, kKStep);
        const int splits = (Bp + gw.k_split - 1) / gw.k_split;
        gw.P = s->P;
        e = gemm<kWGrad>(gw, splits, st);
        if (e != hipSuccess) break;
        float* gW = s->g + s->off[l];
        float* gb = gW + (int64_t)s->fin[l] * s->fout[l];
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk((int64_t)s->fin[l] * s->fout[l], 256)), dim3(256), 0, st, s->P,
                           splits, s->Kp[l], s->Np[l], s->fin[l], s->fout[l], gW);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_bias_grad, dim3(s->fout[l]), dim3(256), 0, st, dZt, Bp, s->fout[l], gb);
        e = hipGetLastError();
        if (e != hipSuccess || l == 0) break;
        // backward data: dZ_{l-1} = (dZ_l W_l^T) * silu'(Z_{l-1})
        GemmArgs gd{};
        gd.A = dZ;
        gd.lda = s->Np[l];
        gd.B = s->Wk[l];
        gd.ldb = s->Np[l];
        gd.M = Bp;
        gd.N = s->Kp[l];
        gd.K = s->Np[l];
        gd.Z = s->Zs[l - 1];
        gd.ldz = s->Np[l - 1];
        gd.H = dN;
        gd.ldh = s->Kp[l];
        gd.Ht = dNt;
        gd.ldt = Bp;
        e = gemm<kBwdData>(gd, 1, st);
        std::swap(dZ, dN);
        std::swap(dZt, dNt);
    }
    return e;
}

int32_t mfail(int32_t c, const std::string& m) { return rcx::fail(c, m); }

}  // namespace

extern "C" {

int32_t rcx_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch, rcx_mlp** out)
{
    if (out) *out = nullptr;
    if (!out) return mfail(RCX_E_INVALID, "rcx_mlp_create: null out");
    if (n_in < 1 || n_in > 16 || n_out < 1 || n_out > 64 || depth < 1 || depth > 16 || width < 16 || width > 512 ||
        width % 64 != 0 || max_batch < 1)
        return mfail(RCX_E_UNSUPPORTED,
                     "rcx_mlp_create: needs 1 <= n_in <= 16, 1 <= n_out <= 64, 1 <= depth <= 16, width a multiple of "
                     "64 in [64, 512], max_batch >= 1");
    rcx_mlp* s = new (std::nothrow) rcx_mlp();
    if (!s) return mfail(RCX_E_NOMEM, "rcx_mlp_create: host allocation");
    s->n_in = n_in;
    s->width = width;
    s->depth = depth;
    s->n_out = n_out;
    s->max_batch = max_batch;
    s->Bp_max = rup(max_batch, 64);
    s->n_layers = depth + 1;
    for (int l = 0; l < s->n_layers; ++l) {
        const int fi = l == 0 ? n_in : width, fo = l == s->n_layers - 1 ? n_out : width;
        s->fin.push_back(fi);
        s->fout.push_back(fo);
        s->Kp.push_back(l == 0 ? 16 : width);
        s->Np.push_back(l == s->n_layers - 1 ? 64 : width);
        s->off.push_back(s->n_params);
        s->n_params += (int64_t)fi * fo + fo;
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    const int64_t Bp = s->Bp_max;
    chk(dalloc(s, &s->p, sizeof(float) * s->n_params));
    chk(dalloc(s, &s->g, sizeof(float) * s->n_params));
    chk(dalloc(s, &s->m, sizeof(float) * s->n_params));
    chk(dalloc(s, &s->v, sizeof(float) * s->n_params));
    s->Wk.resize(s->n_layers);
    s->Wt.resize(s->n_layers);
    s->bias.resize(s->n_layers);
    for (int l = 0; l < s->n_layers; ++l) {
        chk(dalloc(s, &s->Wk[l], sizeof(__bf16) * s->Kp[l] * s->Np[l]));
        chk(dalloc(s, &s->Wt[l], sizeof(__bf16) * s->Kp[l] * s->Np[l]));
        chk(dalloc(s, &s->bias[l], sizeof(float) * s->Np[l]));
    }
    s->Hs.resize(s->n_layers);
    s->Hts.resize(s->n_layers);
    s->Zs.resize(s->n_layers - 1);
    for (int l = 0; l < s->n_layers; ++l) {
        chk(dalloc(s, &s->Hs[l], sizeof(__bf16) * Bp * s->Kp[l]));
        chk(dalloc(s, &s->Hts[l], sizeof(__bf16) * Bp * s->Kp[l]));
        if (l < s->n_layers - 1) chk(dalloc(s, &s->Zs[l], sizeof(float) * Bp * s->Np[l]));
    }
    const int64_t wmax = std::max<int64_t>(width, 64);
    chk(dalloc(s, &s->dA, sizeof(__bf16) * Bp * wmax));
    chk(dalloc(s, &s->dAt, sizeof(__bf16) * Bp * wmax));
    chk(dalloc(s, &s->dB, sizeof(__bf16) * Bp * wmax));
    chk(dalloc(s, &s->dBt, sizeof(__bf16) * Bp * wmax));
    chk(dalloc(s, &s->Y, sizeof(float) * Bp * n_out));
    chk(dalloc(s, &s->P, sizeof(float) * kSplits * wmax * wmax));
    chk(dalloc(s, &s->loss_part, sizeof(float) * (Bp * 64 / 256 + 1)));
    chk(hipDeviceSynchronize());
    if (e != hipSuccess) {
        rcx_mlp_destroy(s);
        return mfail(RCX_E_NOMEM, std::string("rcx_mlp_create: ") + hipGetErrorName(e));
    }
    *out = s;
    return RCX_OK;
}

int32_t rcx_mlp_n_params(const rcx_mlp* s, int64_t* n)
{
    if (!s || !n) return mfail(RCX_E_INVALID, "rcx_mlp_n_params: null argument");
    *n = s->n_params;
    return RCX_OK;
}

int32_t rcx_mlp_set_params(rcx_mlp* s, const float* flat_host, int64_t n)
{
    if (!s || !flat_host) return mfail(RCX_E_INVALID, "rcx_mlp_set_params: null argument");
    if (n != s->n_params) return mfail(RCX_E_INVALID, "rcx_mlp_set_params: wrong parameter count");
    RCX_HIP_TRY(hipMemcpy(s->p, flat_host, sizeof(float) * n, hipMemcpyHostToDevice));
    RCX_HIP_TRY(hipMemset(s->m, 0, sizeof(float) * n));
    RCX_HIP_TRY(hipMemset(s->v, 0, sizeof(float) * n));
    s->t = 0;
    RCX_HIP_TRY(refresh_copies(s, nullptr));
    RCX_HIP_TRY(hipDeviceSynchronize());
    return RCX_OK;
}

int32_t rcx_mlp_get_params(const rcx_mlp* s, float* flat_host, int64_t n)
{
    if (!s || !flat_host) return mfail(RCX_E_INVALID, "rcx_mlp_get_params: null argument");
    if (n != s->n_params) return mfail(RCX_E_INVALID, "rcx_mlp_get_params: wrong parameter count");
    RCX_HIP_TRY(hipDeviceSynchronize());
    RCX_HIP_TRY(hipMemcpy(flat_host, s->p, sizeof(float) * n, hipMemcpyDeviceToHost));
    return RCX_OK;
}

int32_t rcx_mlp_forward(rcx_mlp* s, const float* x, float* y, int32_t batch, hipStream_t st)
{
    if (!s || !x || !y) return mfail(RCX_E_INVALID, "rcx_mlp_forward: null argument");
    if (batch < 1) return mfail(RCX_E_INVALID, "rcx_mlp_forward: batch must be >= 1");
    for (int32_t b0 = 0; b0 < batch; b0 += s->max_batch) {
        const int32_t B = std::min(s->max_batch, batch - b0);
        RCX_HIP_TRY(forward(s, x + (int64_t)b0 * s->n_in, y + (int64_t)b0 * s->n_out, B, rup(B, 64), st));
    }
    return RCX_OK;
}

int32_t rcx_mlp_gradients(rcx_mlp* s, const float* x, const float* y_ref, int32_t batch, float* grad, float* loss_host,
                          hipStream_t st)
{
    if (!s || !x || !y_ref || !loss_host) return mfail(RCX_E_INVALID, "rcx_mlp_gradients: null argument");
    if (batch < 1 || batch > s->max_batch) return mfail(RCX_E_INVALID, "rcx_mlp_gradients: batch out of range");
    const int32_t Bp = rup(batch, 64);
    RCX_HIP_TRY(forward(s, x, s->Y, batch, Bp, st));
    int nlb = 0;
    RCX_HIP_TRY(backward(s, y_ref, batch, Bp, &nlb, st));
    if (grad) RCX_HIP_TRY(hipMemcpyAsync(grad, s->g, sizeof(float) * s->n_params, hipMemcpyDeviceToDevice, st));
    std::vector<float> lp(nlb);
    RCX_HIP_TRY(hipMemcpyAsync(lp.data(), s->loss_part, sizeof(float) * nlb, hipMemcpyDeviceToHost, st));
    RCX_HIP_TRY(hipStreamSynchronize(st));
    double sum = 0.0;
    for (float v : lp) sum += v;
    *loss_host = (float)(sum / ((double)batch * s->n_out));
    return RCX_OK;
}

int32_t rcx_mlp_train_step(rcx_mlp* s, const float* x, const float* y_ref, int32_t batch, float lr, float* loss_host,
                           hipStream_t st)
{
    int32_t rc = rcx_mlp_gradients(s, x, y_ref, batch, nullptr, loss_host, st);
    if (rc != RCX_OK) return rc;
    s->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)s->t), c2 = 1.0f - std::pow(b2, (float)s->t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(s->n_params, 256)), dim3(256), 0, st, s->p, s->g, s->m, s->v, s->n_params,
                       lr, b1, b2, 1e-8f, c1, c2);
    RCX_HIP_TRY(hipGetLastError());
    RCX_HIP_TRY(refresh_copies(s, st));
    return RCX_OK;
}

int32_t rcx_mlp_destroy(rcx_mlp* s)
{
    if (!s) return RCX_OK;
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
    return RCX_OK;
}

}  // extern "C"
