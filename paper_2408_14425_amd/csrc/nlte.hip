// nlte.hip -- the non-LTE iteration around the radiance-cascades formal
// solution (Osborne & Sannikov, arXiv:2408.14425, Sec. 3.3) on gfx950.
//
// Per iteration:
//   k_synth      populations (FP64) -> per-cell line records and continuum
//                fields (FP32) for the march, and per-cell records for the
//                rate epilogue;
//   march        every cascade top-down per 16-wavelength batch; line batches
//                evaluate the Doppler-shifted Voigt opacity per ray step
//                (Sec. 3.2: velocity-dependent terms per ray, observer frame);
//   cascade 0    the march kernel with a rate epilogue: Psi*, I_eff and the
//                preconditioned rate coefficients per (cell, direction,
//                wavelength), reduced over the wavefront (16 wavelengths x 4
//                directions of one cell) without atomics;
//   k_rates_sum  per-transition sums over its batches, in a fixed order;
//   k_stat_eq    Gamma per cell in FP64, diagonal from conservation, one row
//                replaced by particle conservation, Gaussian elimination with
//                partial pivoting; the max relative change is reduced with an
//                integer atomic max on the (non-negative) FP64 bit pattern.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "march_rows.h"

namespace rcx {
namespace nl {

using march::kBlock;
using march::kLB;

// CODATA 2018, SI
constexpr double kH = 6.62607015e-34;
constexpr double kC = 2.99792458e8;
constexpr double kKB = 1.380649e-23;
constexpr double kMe = 9.1093837015e-31;
constexpr double kQe = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kLog2eD = 1.4426950408889634074;

constexpr int kMaxL = RCX_NLTE_MAX_LEVELS;
constexpr int kMaxT = RCX_NLTE_MAX_LINES + RCX_NLTE_MAX_CONTS;

// One transition as the device kernels see it.
struct Trans {
    int32_t kind;   // 0 line, 1 continuum
    int32_t i, j;   // lower, upper level
    int32_t line;   // line index (kind 0) or continuum index (kind 1)
    double nu0;     // line centre / edge frequency [Hz]
    double sigma;   // line: e^2 f / (4 eps0 m_e c) [m^2 Hz]; continuum: alpha at the edge [m^2]
    double gr;      // g_i / g_j
    double U0;      // line: 2 h nu0^3 / c^2
    double gamma;   // line: natural damping [1/s]
    double q;       // collisional de-excitation coefficient [m^3/s]
};

struct AtomDev {
    int32_t nl, nt, n_lines, n_conts;
    double E[kMaxL];  // [J]
    double g[kMaxL];
    double mass;      // [kg]
    Trans t[kMaxT];
};

// ---------------------------------------------------------------- Voigt table
// H(a, x) on a uniform grid a in [0, a_max] (kNa nodes), x in [0, kXTab]
// (kNx nodes); each entry holds the pair {H(x_i), H(x_{i+1})} so one 8-byte
// load gives both x neighbours. Beyond kXTab the asymptotic series
// H ~ a / (sqrt(pi) x^2) (1 + 3/(2x^2) + 15/(4x^4) + 105/(8x^6) + 945/(16x^8))
// is used (relative truncation < 1e-7 there; exp(-x^2) < 1e-27).
constexpr int kNa = 41;
constexpr double kXTab = 8.0;
constexpr int kNx = 4097;  // dx = 1/512

struct VoigtTab {
    const float2* tab;
    float inv_da;
    float inv_dx;
};

__device__ __forceinline__ float voigt_lookup(const VoigtTab& V, float a, float ax)
{
    const float fa = fminf(fmaxf(a * V.inv_da, 0.0f), (float)(kNa - 1) - 1e-3f);
    const int ia = (int)fa;
    const float wa = fa - (float)ia;
    const float fx = fminf(fmaxf(ax * V.inv_dx, 0.0f), (float)(kNx - 1) - 1e-3f);
    const int ix = (int)fx;
    const float wx = fx - (float)ix;
    const float2 p0 = V.tab[ia * kNx + ix];
    const float2 p1 = V.tab[(ia + 1) * kNx + ix];
    const float h0 = fmaf(wx, p0.y - p0.x, p0.x);
    const float h1 = fmaf(wx, p1.y - p1.x, p1.x);
    const float ht = fmaf(wa, h1 - h0, h0);
    const float r = 1.0f / fmaxf(ax * ax, 1.0f);
    const float ser = 1.0f + r * (1.5f + r * (3.75f + r * (13.125f + r * 59.0625f)));
    const float hs = a * 0.5641895835477563f * r * ser;  // a / sqrt(pi) / x^2 * series
    return ax < (float)kXTab ? ht : hs;
}

// Fill: H(a, x) = pi^{-1/2} int_0^inf exp(-a t - t^2/4) cos(x t) dt (the
// Fourier form of the Voigt function), integrated over [0, 13] (the
// integrand is below 1e-18 beyond) with 8-point Gauss-Legendre on 104
// panels of width 1/8, in FP64.
__device__ double voigt_fourier(double a, double x)
{
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double h = 0.125;
    double acc = 0.0;
    for (int p = 0; p < 104; ++p) {
        const double c = (p + 0.5) * h;
        for (int q = 0; q < 4; ++q) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double t = c + sgn * 0.5 * h * gx[q];
                acc += gw[q] * exp(-a * t - 0.25 * t * t) * cos(x * t);
            }
        }
    }
    return acc * 0.5 * h / sqrt(kPi);
}

__global__ void k_voigt_fill(float2* tab, double da, double dx)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)kNa * kNx) return;
    const int ia = (int)(idx / kNx), ix = (int)(idx % kNx);
    const double a = ia * da;
    const double h0 = voigt_fourier(a, ix * dx);
    const double h1 = (ix + 1 < kNx) ? voigt_fourier(a, (ix + 1) * dx) : h0;
    tab[idx] = make_float2((float)h0, (float)h1);
}

__global__ void k_voigt_eval(VoigtTab V, int32_t n, const float* a, const float* x, float* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = voigt_lookup(V, a[i], fabsf(x[i]));
}

// Compact profile table for the march, copied into LDS by every workgroup:
// {H(a_k, x_i), dH/dx(a_k, x_i) * dxc} at a_k = k da (k < n_a <= kNacMax)
// and x_i = i dxc, dxc = 1/32 on [0, kXTab]; cubic Hermite in x (error
// below 3e-8 of H(0, 0)), linear in a (error below da^2 / 4 of H(0, 0)).
// dH/dx = 2 (a L - x H) with L(a, x) = Im w(x + i a) the Faraday-Voigt
// function, from the same Fourier integral:
// L = pi^{-1/2} int_0^inf exp(-a t - t^2/4) sin(x t) dt.
constexpr int kNxc = 257;
constexpr int kNacMax = 9;
constexpr float kInvDxc = 32.0f;
constexpr int kCompactBytes = kNacMax * kNxc * 8;

__device__ void voigt_fourier2(double a, double x, double& H, double& L)
{
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double h = 0.125;
    double ac = 0.0, as = 0.0;
    for (int p = 0; p < 104; ++p) {
        const double c = (p + 0.5) * h;
        for (int q = 0; q < 4; ++q) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double t = c + sgn * 0.5 * h * gx[q];
                const double e = gw[q] * exp(-a * t - 0.25 * t * t);
                double sn, cs;
                sincos(x * t, &sn, &cs);
                ac += e * cs;
                as += e * sn;
            }
        }
    }
    H = ac * 0.5 * h / sqrt(kPi);
    L = as * 0.5 * h / sqrt(kPi);
}

__global__ void k_voigt_fill_compact(float2* tab, int32_t n_a, double da)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_a * kNxc) return;
    const int ia = idx / kNxc, ix = idx % kNxc;
    const double a = ia * da, x = ix / (double)kInvDxc;
    double H, L;
    voigt_fourier2(a, x, H, L);
    tab[idx] = make_float2((float)H, (float)(2.0 * (a * L - x * H) / (double)kInvDxc));
}

// Cubic Hermite at fraction t between nodes q0, q1 = {value, derivative * dxc}.
__device__ __forceinline__ float hermite(float t, float2 q0, float2 q1)
{
    const float t2 = t * t;
    const float h01 = t2 * fmaf(-2.0f, t, 3.0f);  // t^2 (3 - 2t)
    const float h00 = 1.0f - h01;
    const float tm1 = t - 1.0f;
    const float h10 = t * tm1 * tm1;              // t (t - 1)^2
    const float h11 = t2 * tm1;                   // t^2 (t - 1)
    return fmaf(h00, q0.x, fmaf(h10, q0.y, fmaf(h01, q1.x, h11 * q1.y)));
}

// The asymptotic series of H beyond kXTab, without its factor a / sqrt(pi):
// q (1 + 3/2 q + 15/4 q^2 + 105/8 q^3 + 945/16 q^4), q = 1 / x^2.
__device__ __forceinline__ float voigt_wing_series(float q)
{
    return q * fmaf(q, fmaf(q, fmaf(q, fmaf(q, 59.0625f, 13.125f), 3.75f), 1.5f), 1.0f);
}

// H(a, ax) from the LDS table; fa = a / da (inside [0, n_a - 1)),
// a_sqrtpi = a / sqrt(pi) for the asymptotic series beyond kXTab.
__device__ __forceinline__ float voigt_compact(const float2* __restrict__ tab, float fa, float a_sqrtpi, float ax)
{
    const int ia = (int)fa;
    const float wa = __builtin_amdgcn_fractf(fa);
    const float fx = fminf(ax * kInvDxc, (float)(kNxc - 1) - 1e-3f);
    const int ix = (int)fx;
    const float t = __builtin_amdgcn_fractf(fx);
    const float2* p = tab + ia * kNxc + ix;
    const float H0 = hermite(t, p[0], p[1]);
    const float H1 = hermite(t, p[kNxc], p[kNxc + 1]);
    const float ht = fmaf(wa, H1 - H0, H0);
    return ax < (float)kXTab ? ht : a_sqrtpi * voigt_wing_series(__builtin_amdgcn_rcpf(ax * ax));
}

// Small damping. H is harmonic in (x, a), so about a = 0
//   H(a, x) = e^{-x^2} (1 + a^2 (1 - 2 x^2)) - (2 a / sqrt(pi)) g(x) + R,
//   g(x) = 1 - 2 x F(x) = F'(x), F = Dawson's function,
// from H(0, x) = e^{-x^2}, dH/da(0, x) = -(2/sqrt(pi)) g(x) and
// d2H/da2 = -d2H/dx2; the remainder R = (a^3/3 sqrt(pi)) g''(x) + O(a^4)
// is below 0.76 a^3 of H(0, 0) and below about a^2 / 4 of H at any x (its
// relative size peaks where e^{-x^2} and the a term are equal, near x = 3).
// Used when every cell has a <= kSmallAMax (remainder below 7e-6 of H). The
// table holds {g_i, g_{i+1} - g_i} at x_i = i / kInvDg on [0, kXTab],
// linear in x (error below 6e-6 of H where the a term matters, x > 2);
// beyond it g is -1/2 times the series above.
constexpr double kSmallAMax = 5e-3;
constexpr float kInvDg = 256.0f;
constexpr int kNg = 8 * 256 + 1;
static_assert(kNg <= kNacMax * kNxc, "the g table shares the compact table's buffers");

// kCore: the caller knows ax < kXTab (no series).
template <bool kCore = false>
__device__ __forceinline__ float voigt_small_a(const float2* __restrict__ gtab, float a2, float ca, float ax)
{
    const float x2 = ax * ax;
    const float e = __builtin_amdgcn_exp2f(-x2 * march::kLog2e);
    // with ax < kXTab (kCore) ax * kInvDg (a power of two: exact) is below
    // kNg - 1, so the index needs no clamp
    const float fx = kCore ? ax * kInvDg : fminf(ax * kInvDg, (float)(kNg - 1) - 1e-3f);
    const float2 q = gtab[(int)fx];
    const float gt = fmaf(__builtin_amdgcn_fractf(fx), q.y, q.x);
    const float g = (!kCore && ax >= (float)kXTab) ? -0.5f * voigt_wing_series(__builtin_amdgcn_rcpf(x2)) : gt;
    return fmaf(e, fmaf(a2, fmaf(-2.0f, x2, 1.0f), 1.0f), -ca * g);
}

// rx H(a, x) from a staged record's coefficients A = rx (1 + a^2), B = -2 rx
// a^2 and C = rx 2a/sqrt(pi) (rx = the step's opacity scale times its
// length): e^{-x^2} (A + B x^2) - C g(x), the products with rx taken once
// per segment when the record is staged.
template <bool kCore = false>
__device__ __forceinline__ float voigt_small_a_rx(const float2* __restrict__ gtab, float A, float B, float C, float ax)
{
    const float x2 = ax * ax;
    const float e = __builtin_amdgcn_exp2f(-x2 * march::kLog2e);
    const float fx = kCore ? ax * kInvDg : fminf(ax * kInvDg, (float)(kNg - 1) - 1e-3f);
    const float2 q = gtab[(int)fx];
    const float gt = fmaf(__builtin_amdgcn_fractf(fx), q.y, q.x);
    const float g = (!kCore && ax >= (float)kXTab) ? -0.5f * voigt_wing_series(__builtin_amdgcn_rcpf(x2)) : gt;
    return fmaf(e, fmaf(B, x2, A), -C * g);
}

// g(x) = 1 - 2x F(x), with L(0, x) = (2 / sqrt(pi)) F(x) from the Fourier integral.
__device__ double dawson_g(double x)
{
    double H, L;
    voigt_fourier2(0.0, x, H, L);
    return 1.0 - x * sqrt(kPi) * L;
}

__global__ void k_dawson_fill(float2* tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNg) return;
    const double g0 = dawson_g(i / (double)kInvDg), g1 = dawson_g((i + 1) / (double)kInvDg);
    tab[i] = make_float2((float)g0, (float)(g1 - g0));
}

// The march's profile at arbitrary (a, x), for checking the compact table.
__global__ __launch_bounds__(256) void k_voigt_eval_compact(const float2* __restrict__ tabc, int32_t n_a, float inv_da,
                                                            float da_sqrtpi, int32_t small_a, int32_t n, const float* a,
                                                            const float* x, float* out)
{
    __shared__ float2 tab[kNacMax * kNxc];
    const int n_tab = small_a ? kNg : n_a * kNxc;
    for (int i = threadIdx.x; i < n_tab; i += blockDim.x) tab[i] = tabc[i];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        if (small_a) {
            out[i] = voigt_small_a(tab, a[i] * a[i], (float)(2.0 / sqrt(kPi)) * a[i], fabsf(x[i]));
        } else {
            const float fa = fminf(a[i] * inv_da, (float)(n_a - 1) - 1e-3f);
            out[i] = voigt_compact(tab, fa, fa * da_sqrtpi, fabsf(x[i]));
        }
    }
}

// ------------------------------------------------------------ static data
// Per cell, from T, ne, ntot (FP64): Saha-Boltzmann populations, collisional
// rates, 1/v_th, line damping a and sigma/(sqrt(pi) dnu_D), and for each
// continuum log2(n_i*/n_c*) and h/(k T) log2(e).
struct StaticOut {
    double* lte;       // [nl][ncell]
    double* cup;       // [nt][ncell]
    double* cdn;       // [nt][ncell]
    float* inv_vth;    // [ncell]
    float* adamp;      // [n_lines][ncell]
    float* sphi;       // [n_lines][ncell]
    float* lratio;     // [n_conts][ncell]
    float* hkt2;       // [ncell]
    unsigned int* amax_bits;  // max damping over cells and lines (float bits)
};

__global__ void k_static(AtomDev A, int64_t ncell, const double* __restrict__ T, const double* __restrict__ ne,
                         const double* __restrict__ ntot, StaticOut o)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float amax = 0.0f;
    if (c < ncell) {
        const double t = T[c], e = ne[c], n = ntot[c];
        const double kT = kKB * t;
        double rel[kMaxL];
        double sum = 0.0;
        const int cl = A.nl - 1;  // continuum level
        for (int l = 0; l < cl; ++l) {
            rel[l] = A.g[l] / A.g[0] * exp(-(A.E[l] - A.E[0]) / kT);
            sum += rel[l];
        }
        const double saha = 2.0 * pow(2.0 * kPi * kMe * kT / (kH * kH), 1.5) / e;
        rel[cl] = A.g[cl] / A.g[0] * saha * exp(-(A.E[cl] - A.E[0]) / kT);
        sum += rel[cl];
        for (int l = 0; l < A.nl; ++l) o.lte[(int64_t)l * ncell + c] = rel[l] / sum * n;
        const double vth = sqrt(2.0 * kKB * t / A.mass);
        o.inv_vth[c] = (float)(1.0 / vth);
        for (int k = 0; k < A.nt; ++k) {
            const Trans& tr = A.t[k];
            const double cd = e * tr.q / sqrt(t / 1e4);
            o.cdn[(int64_t)k * ncell + c] = cd;
            o.cup[(int64_t)k * ncell + c] = cd * rel[tr.j] / rel[tr.i];
            if (tr.kind == 0) {
                const double dnuD = tr.nu0 * vth / kC;
                const float a = (float)(tr.gamma / (4.0 * kPi * dnuD));
                o.adamp[(int64_t)tr.line * ncell + c] = a;
                o.sphi[(int64_t)tr.line * ncell + c] = (float)(tr.sigma / (sqrt(kPi) * dnuD));
                amax = fmaxf(amax, a);
            } else {
                o.lratio[(int64_t)tr.line * ncell + c] = (float)log2(rel[tr.i] / rel[tr.j]);
            }
        }
        o.hkt2[c] = (float)(kH / kT * kLog2eD);
    }
    // block max of the damping, then one atomic per block (non-negative floats
    // order like their bit patterns)
    __shared__ float red[256];
    red[threadIdx.x] = amax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(o.amax_bits, __float_as_uint(red[0]));
}

// out = a + b per cell (the pressure P / (k T) = n_Htot + n_e, A_tot = 1).
__global__ void k_sum2(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

// -------------------------------------------------------------- synthesis
// Lines: rec[line][c] = {kappa (optical depth per cell at H = 1, log2 units),
// S_line, a in Voigt-table units (a / da), 1/v_th}, with kappa = sigma/(sqrt(pi) dnu_D) (n_i - g_i/g_j n_j)
// voxel and S_line = U0 (g_i/g_j) n_j / (n_i - g_i/g_j n_j) (complete
// redistribution: eta and chi share the profile); epi[line][c] = {n_i, n_j,
// sigma/(sqrt(pi) dnu_D), 0}. Continua: epi[cont][c] = {n_i, n_c,
// log2(n_i*/n_c*), h/(kT) log2 e}; their per-wavelength fields come from
// k_synth_cont.
constexpr float kChiFloor = 1e-20f;  // optical depth per cell, natural units

struct SynthArgs {
    const double* pops;  // [nl][ncell]
    const float* inv_vth;
    const float* adamp;
    const float* sphi;
    const float* lratio;
    const float* hkt2;
    float4* line_rec;    // [n_lines][ncell]
    float4* epi_rec;     // [n_trans][ncell]
    double voxel;
    float inv_da;        // 1 / (damping step of the march's profile table)
    int32_t n_a;         // damping nodes of that table
};

__global__ void k_synth(AtomDev A, int64_t ncell, SynthArgs s)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int k = 0; k < A.nt; ++k) {
        const Trans& tr = A.t[k];
        const double ni = s.pops[(int64_t)tr.i * ncell + c];
        const double nj = s.pops[(int64_t)tr.j * ncell + c];
        if (tr.kind == 0) {
            const double sp = s.sphi[(int64_t)tr.line * ncell + c];
            const double dn = ni - tr.gr * nj;
            double kap = sp * dn * s.voxel;  // natural units per cell
            double S = tr.U0 * tr.gr * nj / dn;
            if (!(kap >= kChiFloor)) {  // no (or inverted) line opacity: keep the emission finite
                S = tr.U0 * tr.gr * nj * sp * s.voxel / kChiFloor;
                kap = kChiFloor;
            }
            const float fa = fminf(s.adamp[(int64_t)tr.line * ncell + c] * s.inv_da, (float)(s.n_a - 1) - 1e-3f);
            s.line_rec[(int64_t)tr.line * ncell + c] = make_float4((float)(kap * kLog2eD), (float)S, fa, s.inv_vth[c]);
            s.epi_rec[(int64_t)k * ncell + c] = make_float4((float)ni, (float)nj, (float)sp, 0.0f);
        } else {
            s.epi_rec[(int64_t)k * ncell + c] =
                make_float4((float)ni, (float)nj, s.lratio[(int64_t)tr.line * ncell + c], s.hkt2[c]);
        }
    }
}

// Continuum batch b: F[b][c][l] = {kappa (log2 units per cell), S} with
// chi = alpha (n_i - n_c (n_i*/n_c*) e^{-h nu/kT}), eta = (2 h nu^3/c^2) alpha
// n_c (n_i*/n_c*) e^{-h nu/kT}, alpha = alpha0 (nu_edge/nu)^3 (FP64).
struct ContBatch {
    int32_t trans;
    int32_t n;        // valid wavelengths in the batch
    double nu[kLB];
};

__global__ void k_synth_cont(AtomDev A, int64_t ncell, const double* __restrict__ pops, const double* __restrict__ T,
                             ContBatch cb, const float* lratio, double voxel, float2* __restrict__ Fb,
                             unsigned int* __restrict__ smax_b)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = idx < ncell * kLB;  // no early return: the block reduces below
    const int64_t c = in ? idx / kLB : 0;
    const int l = (int)(idx % kLB);
    float2 v = make_float2(0.0f, 0.0f);
    if (in && l < cb.n) {
        const Trans& tr = A.t[cb.trans];
        const double ni = pops[(int64_t)tr.i * ncell + c];
        const double nc = pops[(int64_t)tr.j * ncell + c];
        const double nu = cb.nu[l];
        const double alpha = tr.sigma * pow(tr.nu0 / nu, 3.0);
        const double lr = lratio[(int64_t)tr.line * ncell + c];
        const double stim = exp2(lr - kH * nu / (kKB * T[c]) * kLog2eD);  // (n_i*/n_c*) e^{-h nu / kT}
        const double chi = alpha * (ni - nc * stim) * voxel;
        const double eta = 2.0 * kH * nu * nu * nu / (kC * kC) * alpha * nc * stim * voxel;
        if (chi >= kChiFloor)
            v = make_float2((float)(chi * kLog2eD), (float)(eta / chi));
        else
            v = make_float2(kChiFloor * (float)kLog2eD, (float)(eta / kChiFloor));
    }
    if (in) Fb[idx] = v;
    if (smax_b) {
        // per-wavelength max of S over the 16 cells of this block (lanes l,
        // l + 16, ... hold wavelength l), then one atomic per wavelength
        float m = v.y;
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        __shared__ float red[256 / 64][kLB];
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (lane < kLB) red[w][lane] = m;
        __syncthreads();
        if (threadIdx.x < kLB) {
            float r = red[0][threadIdx.x];
            for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = fmaxf(r, red[q][threadIdx.x]);
            atomicMax(&smax_b[threadIdx.x], __float_as_uint(r));
        }
    }
}

// Sparse: zero the opacity scale and source function of the line records
// ([n_lines][ncell] float4 {kappa, S, ...}) at unflagged cells.
__global__ void k_mask_line_rec(float4* __restrict__ rec, const uint8_t* __restrict__ mask, int64_t ncell,
                                int32_t n_lines)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)n_lines * ncell && !mask[i % ncell]) {
        rec[i].x = 0.0f;
        rec[i].y = 0.0f;
    }
}

// Max over cells of a line's source function (every wavelength of a line
// batch shares S_line), into all 16 entries of the batch's smax.
__global__ void k_smax_line(int64_t ncell, const float4* __restrict__ rec, unsigned int* __restrict__ smax_b)
{
    __shared__ float red[256];
    float m = 0.0f;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, rec[c].y);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x < kLB) atomicMax(&smax_b[threadIdx.x], __float_as_uint(red[0]));
}

__global__ void k_zero_u32n(unsigned int* p, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------ line march op
// Opacity of a line batch at one ray step: x = (u_l + w . v) / v_th (the
// profile of a ray looking along w, photons travelling along -w, in the
// observer's frame), chi = kappa H(a, |x|), S = S_line. kSmallA selects the
// profile: the expansion in a (voigt_small_a, record z = a) or the compact
// table in (a, x) (voigt_compact, record z = a / da).
//
// kG > 1: each lane marches wavelength l of kG consecutive batches of the
// same line (slot w's velocity offsets at u_b + w u_stride): one walk and one
// staged record per segment serve all of them, and the cascades hold kG
// slots (StoreEpiSlots / StoreF16EpiSlots).
template <bool kSmallA, int kG = 1>
struct LineOpT {
    const float4* rec;  // [ncell]
    const float2* vel;  // [ncell]
    const float2* tabc; // profile table [n_a][kNxc] (global; copied to LDS)
    int32_t n_a;
    const float* u_b;   // [16] velocity offsets of the batch's wavelengths [m/s]
    int32_t u_stride = 0;  // kG > 1: elements from one slot's offsets to the next's
    uint32_t ncell;
    float da_sqrtpi;    // damping step of the table / sqrt(pi)
    float u[kG], wx, wz;
    float vscale = 1.0f;  // velocity projection: sin(theta) of an inclined ray (Sec. 3.1), 1 in the plane
    const float2* tab;  // the LDS copy
    // the cell record and velocity are the same for all wavelength lanes;
    // with kSmallA the entry also carries {a^2, 2a / sqrt(pi)} and holds
    // (w . v) / v_th in place of the velocity's x component
    static constexpr int kW = kG;
    static constexpr bool kStaged = true;
    struct Stage {
        float4 r;
        float2 v;
        float2 p;
    };
    using Raw = Stage;
    struct StageIn {
        float4 r;
        float2 v;
    };
    static constexpr int kSmemBytes = kSmallA ? kNg * 8 : kCompactBytes;
    __device__ __forceinline__ void init_shared(float2* smem)
    {
        const int n_tab = kSmallA ? kNg : n_a * kNxc;
        for (int i = threadIdx.x; i < n_tab; i += blockDim.x) smem[i] = tabc[i];
        tab = smem;
    }
    // segment entries keep the cell index (the step loop reads the staged
    // record); a null entry has ds = 0
    static constexpr uint32_t kNullKey = 0u;
    __device__ __forceinline__ uint32_t key(uint32_t cell) const { return cell; }
    __device__ __forceinline__ StageIn stage_load(uint32_t cell) const { return StageIn{rec[cell], vel[cell]}; }
    // the entry of a segment of length ds: its opacity scale times ds, so
    // the profile times it is the step's optical depth
    __device__ __forceinline__ Stage stage_make(const StageIn& in, float ds) const
    {
        Stage st;
        st.r = in.r;
        st.r.x = in.r.x * ds;
        st.v = in.v;
        // with the expansion in a: r.x = rx (1 + a^2), p = {-2 rx a^2, rx 2a /
        // sqrt(pi)} (voigt_small_a_rx)
        if constexpr (kSmallA) {
            const float rx = st.r.x, rxa2 = rx * (in.r.z * in.r.z);
            st.r.x = rx + rxa2;
            st.p = make_float2(-2.0f * rxa2, rx * ((float)(2.0 / sqrt(kPi)) * in.r.z));
        } else {
            st.p = make_float2(0.0f, 0.0f);
        }
        if constexpr (kSmallA) st.v.x = (wx * in.v.x + wz * in.v.y) * in.r.w;  // (w . v) / v_th
        return st;
    }
    __device__ __forceinline__ void init(int l)
    {
#pragma unroll
        for (int w = 0; w < kG; ++w) u[w] = u_b[l + w * u_stride];
    }
    __device__ __forceinline__ void begin_ray(double dwx, double dwz)
    {
        wx = (float)dwx * vscale;
        wz = (float)dwz * vscale;
    }
    // H(a, |x|), x = (u + w . v) / v_th, from a record and a velocity
    __device__ __forceinline__ float profile(const float4& r, const float2& v) const
    {
        const float ax = fabsf((u[0] + wx * v.x + wz * v.y) * r.w);
        if constexpr (kSmallA) return voigt_small_a(tab, r.z * r.z, (float)(2.0 / sqrt(kPi)) * r.z, ax);
        return voigt_compact(tab, r.z, r.z * da_sqrtpi, ax);
    }
    __device__ __forceinline__ float2 resolve(const Raw& raw, float uw) const
    {
        if constexpr (kSmallA) {
            const float ax = fabsf(fmaf(uw, raw.r.w, raw.v.x));
            return make_float2(voigt_small_a_rx(tab, raw.r.x, raw.p.x, raw.p.y, ax), raw.r.y);
        }
        const float ax = fabsf((uw + wx * raw.v.x + wz * raw.v.y) * raw.r.w);
        return make_float2(raw.r.x * voigt_compact(tab, raw.r.z, raw.r.z * da_sqrtpi, ax), raw.r.y);
    }
    // {chi, S} of a group of 4 staged steps for slot w (the batch of u[w]).
    // With the expansion in a, the series beyond kXTab is evaluated only when
    // a lane of the wavefront needs it (the line-core batches never do).
    __device__ __forceinline__ void resolve4(const Raw (&raw)[4], float2 (&f)[4], int w) const
    {
        const float uw = u[w];
        if constexpr (kSmallA) {
            float ax[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) ax[q] = fabsf(fmaf(uw, raw[q].r.w, raw[q].v.x));
            // one compare of the group's largest |x| (a NaN lane takes the
            // core path, whose index conversion maps it to entry 0)
            const float ax_max = fmaxf(fmaxf(ax[0], ax[1]), fmaxf(ax[2], ax[3]));
            if (__ballot(ax_max >= (float)kXTab) != 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    f[q] = make_float2(voigt_small_a_rx(tab, raw[q].r.x, raw[q].p.x, raw[q].p.y, ax[q]), raw[q].r.y);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    f[q] = make_float2(voigt_small_a_rx<true>(tab, raw[q].r.x, raw[q].p.x, raw[q].p.y, ax[q]),
                                       raw[q].r.y);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) f[q] = resolve(raw[q], uw);
        }
    }
};
using LineOp = LineOpT<false>;
using LineOpSmallA = LineOpT<true>;

// ----------------------------------------------------------- rate epilogue
// At cascade 0 every wavefront holds the 4 directions (rows) x 16
// wavelengths of one cell. Each lane forms, with I the merged radiance,
//   Psi* = l (1 - e^{-tau}) / tau,  tau = chi_t l  (l = distance from the
//          cell centre to its edge along the ray, m)
//   I_eff = I - Psi* eta_t
//   up   = W V_ij I_eff,   down = W (V_ji I_eff + U_ji (1 - chi_t Psi*))
// (W = 4 pi dnu/(h nu) / N_0 per lane, 0 on padding lanes); the wavefront sum
// goes to part[c] = {up, down}. An inclined ray (Sec. 3.1) crosses the cell
// on a path `path` = 1/sin(theta) times longer, its terms are weighted by
// its quadrature weight `wgt`, and inclinations after the first add to part.
struct RatesEpi {
    float* out;             // merged cascade 0 [rays][16] (for J)
    float2* part;           // [ncell] this batch's rate contributions
    const float4* epi_rec;  // [ncell] of the batch's transition
    const float* W;         // [16]
    const float* nu;        // [16] (continuum batches)
    const float* alpha;     // [16] alpha(nu) (continuum batches)
    const float* U0c;       // [16] 2 h nu^3 / c^2 (continuum batches)
    float gr, U0;           // line: g_i/g_j, 2 h nu0^3 / c^2
    float ell_cells, voxel; // l in cells (the same for all N_0 directions), cell size [m]
    int32_t kind;           // 0 line, 1 continuum
    float path = 1.0f, wgt = 1.0f;
    bool acc = false;

    __device__ __forceinline__ void init(int) {}

    // I is the merged radiance of the ray beyond its own cell: the launch
    // marches [l, t_1) (l the distance from the cell centre to its edge
    // along the ray, where the ray leaves the cell through a corner), and
    // the cell's own part, Psi* eta_t = S (1 - e^{-tau}), is added here.
    // Then I_eff = I_full - Psi* eta_t = e^{-tau} I is formed without the
    // cancellation of two nearly equal FP32 numbers in optically thick
    // cells, and 1 - chi_t Psi* = e^{-tau} likewise.
    template <class Op>
    __device__ __forceinline__ void finish(const march::RayInfo& ri, int l, int lane, float I, const Op& op)
    {
        const int64_t cell = ri.ray / 4;  // cascade 0: ray = cell * 4 + direction
        float up = 0.0f, dn = 0.0f;
        if (ri.active) {
            const float4 e = epi_rec[cell];
            // V_ji = A S2 is never formed on its own: for a far-UV continuum
            // in cool gas alpha (n_i*/n_c*) e^{-h nu/kT} falls below FP32's
            // range (2.5e-48 at 5000 K and half the Lyman edge) while each
            // product with n_c, U0 or W, taken before S2, stays inside it
            float Vij, A, S2, U0x;
            if (kind == 0) {
                const float H = line_profile(op, (uint32_t)cell);
                Vij = e.z * H;
                A = gr * Vij;
                S2 = 1.0f;
                U0x = U0;
            } else {
                Vij = alpha[l];
                A = Vij;
                S2 = __builtin_amdgcn_exp2f(fminf(e.z - nu[l] * e.w, 126.0f));
                U0x = U0c[l];
            }
            const float eta_t = ((e.y * U0x) * A) * S2;
            const float chi_t = e.x * Vij - (e.y * A) * S2;  // [1/m]
            const float ellm = ell_cells * voxel * path;
            const float tau = fmaxf(chi_t * ellm, 0.0f);
            const float T1 = __builtin_amdgcn_exp2f(-tau * march::kLog2e);
            // phi1 = (1 - e^{-tau}) / tau: series below 1/64, direct above
            const float ser = 1.0f - tau * (0.5f - tau * (1.0f / 6.0f - tau * (1.0f / 24.0f)));
            const float phi1 = tau < (1.0f / 64.0f) ? ser : (1.0f - T1) / tau;
            const float psi = ellm * phi1;
            const float ieff = T1 * I;
            out[ri.ray * kLB + l] = fmaf(psi, eta_t, ieff);
            const float stim = chi_t > 0.0f ? T1 : 1.0f - chi_t * psi;
            const float wv = W[l] * wgt;
            up = (wv * Vij) * ieff;
            dn = ((wv * A) * S2) * ieff + (((wv * U0x) * A) * S2) * stim;
        }
        // wavefront sum (fixed butterfly order: deterministic)
        for (int m = 32; m >= 1; m >>= 1) {
            up += __shfl_xor(up, m);
            dn += __shfl_xor(dn, m);
        }
        if (lane == 0 && ri.active) {
            if (acc) {
                const float2 o = part[cell];
                part[cell] = make_float2(o.x + up, o.y + dn);
            } else {
                part[cell] = make_float2(up, dn);
            }
        }
    }

    // H at the cell itself along the ray (only a line op has a profile).
    template <bool K>
    __device__ __forceinline__ float line_profile(const LineOpT<K>& op, uint32_t cell) const
    {
        return op.profile(op.rec[cell], op.vel[cell]);
    }
    __device__ __forceinline__ float line_profile(const march::FieldOp&, uint32_t) const { return 0.0f; }
};

// ------------------------------------------------------------- rate sums
// rates[t][0|1][c] = sum over the batches of transition t (fixed order).
__global__ void k_rates_sum(int64_t ncell, int32_t nt, const int32_t* __restrict__ tb0, const int32_t* __restrict__ tb1,
                            const float2* __restrict__ part, float* __restrict__ rates)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int t = 0; t < nt; ++t) {
        double u = 0.0, d = 0.0;
        for (int b = tb0[t]; b < tb1[t]; ++b) {
            const float2 p = part[(int64_t)b * ncell + c];
            u += p.x;
            d += p.y;
        }
        rates[((int64_t)t * 2 + 0) * ncell + c] = (float)u;
        rates[((int64_t)t * 2 + 1) * ncell + c] = (float)d;
    }
}

// ------------------------------------------------- statistical equilibrium
template <int NL>
__global__ __launch_bounds__(256) void k_stat_eq(AtomDev A, int64_t ncell, const float* __restrict__ rates,
                                                  const double* __restrict__ cup, const double* __restrict__ cdn,
                                                  double* __restrict__ ntot, double* __restrict__ pops,
                                                  unsigned long long* __restrict__ max_change,
                                                  double* __restrict__ ne, const double* __restrict__ p_kt,
                                                  const uint8_t* __restrict__ active)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double change = 0.0;
    // sparse: unflagged cells are held (Sec. 3.5)
    if (c < ncell && (!active || active[c])) {
        double n[NL], G[NL][NL + 1];
        for (int l = 0; l < NL; ++l) {
            n[l] = pops[(int64_t)l * ncell + c];
            for (int m = 0; m <= NL; ++m) G[l][m] = 0.0;
        }
        for (int k = 0; k < A.nt; ++k) {
            const Trans& tr = A.t[k];
            const double up = (double)rates[((int64_t)k * 2 + 0) * ncell + c] + cup[(int64_t)k * ncell + c];
            const double dn = (double)rates[((int64_t)k * 2 + 1) * ncell + c] + cdn[(int64_t)k * ncell + c];
            G[tr.j][tr.i] += up;
            G[tr.i][tr.j] += dn;
        }
        for (int m = 0; m < NL; ++m) {  // diagonal: minus the column sum
            double s = 0.0;
            for (int l = 0; l < NL; ++l)
                if (l != m) s += G[l][m];
            G[m][m] = -s;
        }
        double G0[NL][NL];  // Gamma before the conservation row (charge step)
        for (int l = 0; l < NL; ++l)
            for (int m = 0; m < NL; ++m) G0[l][m] = G[l][m];
        int r = 0;
        for (int l = 1; l < NL; ++l)
            if (n[l] > n[r]) r = l;
        for (int m = 0; m < NL; ++m) G[r][m] = 1.0;
        G[r][NL] = ntot[c];
        // Gaussian elimination with partial pivoting on the augmented matrix
        for (int col = 0; col < NL; ++col) {
            int piv = col;
            for (int l = col + 1; l < NL; ++l)
                if (fabs(G[l][col]) > fabs(G[piv][col])) piv = l;
            if (piv != col)
                for (int m = 0; m <= NL; ++m) {
                    const double t = G[col][m];
                    G[col][m] = G[piv][m];
                    G[piv][m] = t;
                }
            const double inv = 1.0 / G[col][col];
            for (int l = col + 1; l < NL; ++l) {
                const double f = G[l][col] * inv;
                for (int m = col; m <= NL; ++m) G[l][m] -= f * G[col][m];
            }
        }
        double x[NL];
        for (int l = NL - 1; l >= 0; --l) {
            double s = G[l][NL];
            for (int m = l + 1; m < NL; ++m) s -= G[l][m] * x[m];
            x[l] = s / G[l][l];
        }
        if (ne) {
            // charge conservation (Sec. 3.3): one Newton-Raphson step on
            // (n, n_e) with n_e = n_c (the continuum level, hydrogen the
            // only donor). dGamma/dn_e holds the rates proportional to n_e:
            // collisional downward, bound-bound collisional upward and
            // radiative recombination, divided by n_e.
            const double e = ne[c];
            constexpr int cl = NL - 1;
            double D[NL];
            for (int l = 0; l < NL; ++l) D[l] = 0.0;
            for (int k = 0; k < A.nt; ++k) {
                const Trans& tr = A.t[k];
                const double upE = tr.kind == 0 ? cup[(int64_t)k * ncell + c] / e : 0.0;
                const double dnE =
                    (cdn[(int64_t)k * ncell + c] + (tr.kind == 1 ? (double)rates[((int64_t)k * 2 + 1) * ncell + c] : 0.0)) /
                    e;
                D[tr.j] += upE * x[tr.i];
                D[tr.i] -= upE * x[tr.i];
                D[tr.i] += dnE * x[tr.j];
                D[tr.j] -= dnE * x[tr.j];
            }
            int r2 = 0;
            for (int l = 1; l < NL; ++l)
                if (x[l] > x[r2]) r2 = l;
            double M[NL + 1][NL + 2];
            double sx = 0.0;
            for (int l = 0; l < NL; ++l) sx += x[l];
            for (int l = 0; l < NL; ++l) {
                double gx = 0.0;
                for (int m = 0; m < NL; ++m) {
                    M[l][m] = G0[l][m];
                    gx += G0[l][m] * x[m];
                }
                M[l][NL] = D[l];
                M[l][NL + 1] = -gx;
            }
            for (int m = 0; m < NL; ++m) M[r2][m] = 1.0;
            M[r2][NL] = 0.0;
            M[r2][NL + 1] = ntot[c] - sx;
            for (int m = 0; m < NL; ++m) M[NL][m] = 0.0;
            M[NL][cl] = -1.0;
            M[NL][NL] = 1.0;
            M[NL][NL + 1] = x[cl] - e;
            for (int col = 0; col <= NL; ++col) {
                int piv = col;
                for (int l = col + 1; l <= NL; ++l)
                    if (fabs(M[l][col]) > fabs(M[piv][col])) piv = l;
                if (piv != col)
                    for (int m = 0; m <= NL + 1; ++m) {
                        const double t = M[col][m];
                        M[col][m] = M[piv][m];
                        M[piv][m] = t;
                    }
                const double inv = 1.0 / M[col][col];
                for (int l = col + 1; l <= NL; ++l) {
                    const double f = M[l][col] * inv;
                    for (int m = col; m <= NL + 1; ++m) M[l][m] -= f * M[col][m];
                }
            }
            double d[NL + 1];
            for (int l = NL; l >= 0; --l) {
                double s = M[l][NL + 1];
                for (int m = l + 1; m <= NL; ++m) s -= M[l][m] * d[m];
                d[l] = s / M[l][l];
            }
            // the step is taken only if it keeps every population and n_e
            // positive
            bool ok = e + d[NL] > 0.0;
            for (int l = 0; l < NL; ++l) ok = ok && x[l] + d[l] > 0.0;
            if (ok) {
                for (int l = 0; l < NL; ++l) x[l] += d[l];
                const double e1 = e + d[NL];
                change = fmax(change, fabs(e1 - e) / e1);
                ne[c] = e1;
            }
            if (p_kt) {
                // pressure conservation: n_Htot + n_e held at P / (k T)
                // (A_tot = 1), every population scaled with n_Htot
                const double nt0 = ntot[c], nt1 = p_kt[c] - ne[c];
                if (nt1 > 0.0) {
                    const double f = nt1 / nt0;
                    for (int l = 0; l < NL; ++l) x[l] *= f;
                    ntot[c] = nt1;
                    change = fmax(change, fabs(nt1 - nt0) / nt1);
                }
            }
        }
        for (int l = 0; l < NL; ++l) {
            change = fmax(change, fabs(x[l] - n[l]) / fabs(x[l]));
            pops[(int64_t)l * ncell + c] = x[l];
        }
        if (!(change == change)) change = INFINITY;  // NaN: report as non-convergence
    }
    __shared__ double red[256];
    red[threadIdx.x] = change;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(max_change, (unsigned long long)__double_as_longlong(red[0]));
}


// ------------------------------------------------------ warm-start features
// Per cell: {log10 T, log10 ne, |v| [km/s], log10 chi_0 (opacity of line 0 at
// its centre [1/m]), log10 Jbar_t for the first two lines}, Jbar_t the
// profile-weighted mean intensity of line t, sum H(a, u/v_th) dnu J / sum
// H dnu over the line's wavelengths (static profile at the cell); each
// feature standardised with (mean, std).
struct FeatArgs {
    const float* J;        // [n_wave][ncell]
    const double* T;
    const double* ne;
    const float2* vel;
    const float* inv_vth;
    const float* adamp;    // [n_lines][ncell]
    const float4* line_rec;
    const float* u_all;    // [n_wave] velocity offsets (lines)
    const float* dnu_all;  // [n_wave]
    int32_t lam0[2], lam1[2];  // wavelength ranges of lines 0 and 1
    int32_t n_lines;
    float voxel;
    const float* norm;     // [2][6] mean, std
    float* out;            // [ncell][6]
};

__global__ void k_features(int64_t ncell, VoigtTab vt, FeatArgs f)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    float v[6];
    v[0] = log10f((float)f.T[c]);
    v[1] = log10f((float)f.ne[c]);
    const float2 w = f.vel[c];
    v[2] = sqrtf(w.x * w.x + w.y * w.y) * 1e-3f;
    const float kap = f.n_lines > 0 ? f.line_rec[c].x / (f.voxel * march::kLog2e) : 1e-30f;
    v[3] = log10f(fmaxf(kap, 1e-30f));
    for (int t = 0; t < 2; ++t) {
        float num = 0.0f, den = 0.0f;
        if (t < f.n_lines) {
            const float a = f.adamp[(int64_t)t * ncell + c];
            for (int l = f.lam0[t]; l < f.lam1[t]; ++l) {
                const float h = voigt_lookup(vt, a, fabsf(f.u_all[l] * f.inv_vth[c])) * f.dnu_all[l];
                num += h * f.J[(int64_t)l * ncell + c];
                den += h;
            }
        }
        v[4 + t] = log10f(fmaxf(den > 0.0f ? num / den : 0.0f, 1e-35f));
    }
    for (int q = 0; q < 6; ++q) f.out[c * 6 + q] = (v[q] - f.norm[q]) / f.norm[6 + q];
}

// log10(n_l / ntot) per cell, standardised: out[c][l] = (log10 frac - mean_l) / std_l.
__global__ void k_log_departures(int64_t ncell, int32_t nl, const double* __restrict__ pops,
                                 const double* __restrict__ lte, const float* __restrict__ norm, float* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int l = 0; l < nl; ++l) {
        const double b = fmax(pops[(int64_t)l * ncell + c], 1e-300) / fmax(lte[(int64_t)l * ncell + c], 1e-300);
        out[c * nl + l] = ((float)log10(b) - norm[l]) / norm[nl + l];
    }
}

// Populations from predicted standardised log departure coefficients
// y [c][l]: n_l = n_l^LTE 10^{z_l}, z = y std + mean, renormalised to
// sum_l n_l = ntot (FP64).
__global__ void k_pops_from_pred(int64_t ncell, int32_t nl, const float* __restrict__ y, const float* __restrict__ norm,
                                 const double* __restrict__ lte, const double* __restrict__ ntot,
                                 double* __restrict__ pops)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    double n[kMaxL], sum = 0.0;
    for (int l = 0; l < nl; ++l) {
        const double z = (double)y[c * nl + l] * norm[nl + l] + norm[l];
        n[l] = lte[(int64_t)l * ncell + c] * exp10(fmin(z, 30.0));
        sum += n[l];
    }
    for (int l = 0; l < nl; ++l) pops[(int64_t)l * ncell + c] = ntot[c] * n[l] / sum;
}

}  // namespace nl
}  // namespace rcx

// ====================================================================== host

using namespace rcx;
using namespace rcx::nl;

struct rcx_nlte {
    rcx_plan* plan = nullptr;
    AtomDev atom{};
    int32_t n_wave = 0;
    int64_t ncell = 0;
    double voxel = 1.0;
    std::vector<double> lam_nm, dnu;
    std::vector<int32_t> trans;
    struct Batch {
        int32_t trans, lam0, n, cont_slot;  // cont_slot: index of the continuum field slice, or -1
    };
    std::vector<Batch> batches;
    std::vector<int32_t> tb0, tb1;  // batch range of each transition
    int32_t n_cont_batches = 0;
    // device
    float* bconst = nullptr;  // [n_batch][5][16]: W/N0, u, nu, alpha, 2 h nu^3 / c^2
    int32_t* d_tb = nullptr;  // [2][nt]
    double *lte = nullptr, *cup = nullptr, *cdn = nullptr, *T = nullptr, *ntot = nullptr, *ne_copy = nullptr;
    float *inv_vth = nullptr, *adamp = nullptr, *sphi = nullptr, *lratio = nullptr, *hkt2 = nullptr;
    float2* vel = nullptr;
    float4* line_rec = nullptr;
    float4* epi_rec = nullptr;
    float2* Fcont = nullptr;
    float* casc[2] = {nullptr, nullptr};
    // up to `group` consecutive batches of one line march their cascades
    // >= 1 in one pass (LineOpT<_, G>, G = 4 or 2); the cascade buffers then
    // hold `group` slots of casc_slot elements
    int32_t group = 1;
    int64_t casc_slot = 0;
    bool f16 = false;                 // cascades >= 1 stored as scaled FP16
    unsigned int* smax = nullptr;     // [n_batch][16] max S (float bits)
    int32_t* ebias = nullptr;         // [n_batch][16] exponent biases of the 16-bit codes
    float2* part = nullptr;
    float* rates = nullptr;
    unsigned long long* d_max = nullptr;
    unsigned int* d_amax = nullptr;
    unsigned int* d_check = nullptr;  // input check flag (RCX_FLAG_CHECK_INPUT)
    bool check_input = false;
    float2* vtab = nullptr;
    float v_inv_da = 0.0f;
    float2* vtabc = nullptr;  // profile table of the line march
    int32_t n_ac = 2;         // its damping rows (1 with small_a)
    double da_c = 1.0;
    bool small_a = false;     // every a <= kSmallAMax: expansion in a
    int32_t profile_mode = RCX_PROFILE_AUTO;
    // Ng acceleration: order M (0 = off), first after ng_delay iterations,
    // then every ng_period; ring of the last M + 2 iterates
    int32_t ng_order = 0, ng_delay = 0, ng_period = 1;
    // charge conservation: a Newton-Raphson step after each equilibrium
    // step updates ne_copy, and the n_e-dependent static data follow
    int32_t charge = 0;
    // pressure conservation (with charge): n_Htot + n_e held at p_kt
    int32_t pressure = 0;
    double* p_kt = nullptr;  // [ncell] P / (k T) of the atmosphere as set
    int32_t ng_count = 0, ng_head = 0, ng_iter = 0;
    double* ng_hist = nullptr;   // [M + 2][nl][ncell]
    double* ng_part = nullptr;   // [kNgBlocks][kNgSums] partial sums
    double* ng_sums = nullptr;   // [kNgSums]
    bool atm_set = false;
    float* u_all = nullptr;    // [n_wave]
    float* dnu_all = nullptr;  // [n_wave]
    float* Jtmp = nullptr;     // [n_wave][ncell] (warm start)
    float* feat = nullptr;     // [ncell][6]
    float* pred = nullptr;     // [ncell][n_levels]
    float* norms = nullptr;    // [12 + 2 n_levels]
    // measurement: events around every march launch when timing is enabled
    struct Timed {
        int32_t kind;   // 0 line, 1 continuum
        int64_t steps;  // cell steps x wavelengths the launch marches (dense count)
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<Timed> pending;
    std::vector<void*> allocs;
};

namespace {

int32_t nlte_fail(int32_t code, const std::string& m) { return rcx::fail(code, m); }

template <class P>
hipError_t dmalloc(rcx_nlte* s, P** p, size_t bytes)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes < 256 ? 256 : bytes);
    if (e == hipSuccess) s->allocs.push_back(q);
    *p = (P*)q;
    return e;
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }
__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// [2][ncell] planar velocity -> interleaved {vx, vz}
__global__ void k_pack_vel(int64_t ncell, const float* __restrict__ v, float2* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) out[c] = make_float2(v[c], v[ncell + c]);
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class Op, class Epi, class Up>
hipError_t launch_level(const LevelDesc& L0, int32_t nx, int32_t nz, const Op& op, const Epi& epi, const double4* dirs,
                        const Up& up, hipStream_t st)
{
    LevelDesc L = L0;
    if (!set_decode(L)) return hipErrorInvalidValue;  // more rays than 31-bit indices
    const int64_t total = level_launch_rays(L);
    hipLaunchKernelGGL((march::k_march_rows<Op, Epi, Up>), march_grid(total), dim3(kBlock), 0, st, L, nx, nz, op, epi,
                       dirs, up, total);
    return hipGetLastError();
}

// One cascade of one batch: the opacity op (line or field), the epilogue
// (store FP32 / FP16, or the cascade-0 rates) and the reader of the cascade
// above (FP32 or FP16).
template <class Epi, class Up>
hipError_t launch_level_op(int32_t kind, bool small_a, const LevelDesc& L, int32_t nx, int32_t nz, const LineOp& lop,
                           const march::FieldOp& fop, const Epi& epi, const double4* dirs, const Up& up, hipStream_t st)
{
    if (kind != 0) return launch_level(L, nx, nz, fop, epi, dirs, up, st);
    if (small_a) {
        LineOpSmallA sop{};
        sop.rec = lop.rec;
        sop.vel = lop.vel;
        sop.tabc = lop.tabc;
        sop.n_a = lop.n_a;
        sop.u_b = lop.u_b;
        sop.ncell = lop.ncell;
        sop.da_sqrtpi = lop.da_sqrtpi;
        sop.vscale = lop.vscale;
        return launch_level(L, nx, nz, sop, epi, dirs, up, st);
    }
    return launch_level(L, nx, nz, lop, epi, dirs, up, st);
}

// Cascades >= 1 of G batches of one line in one launch (LineOpT<_, G>:
// slot w's velocity offsets u_stride elements after slot w - 1's; G-slot
// epilogue and reader).
template <int G, class Epi, class Up>
hipError_t launch_level_group(bool small_a, const LevelDesc& L, int32_t nx, int32_t nz, const LineOp& lop,
                              int32_t u_stride, const Epi& epi, const double4* dirs, const Up& up, hipStream_t st)
{
    auto fill = [&](auto& op) {
        op.rec = lop.rec;
        op.vel = lop.vel;
        op.tabc = lop.tabc;
        op.n_a = lop.n_a;
        op.u_b = lop.u_b;
        op.u_stride = u_stride;
        op.ncell = lop.ncell;
        op.da_sqrtpi = lop.da_sqrtpi;
        op.vscale = lop.vscale;
    };
    if (small_a) {
        LineOpT<true, G> gop{};
        fill(gop);
        return launch_level(L, nx, nz, gop, epi, dirs, up, st);
    }
    LineOpT<false, G> gop{};
    fill(gop);
    return launch_level(L, nx, nz, gop, epi, dirs, up, st);
}

template <int G>
hipError_t launch_group_casc(bool f16, bool small_a, const LevelDesc& L, int32_t nx, int32_t nz, const LineOp& lop,
                             int32_t u_stride, void* outb, const void* upl, int64_t slot, const int32_t* eb_b,
                             const double4* dirs, hipStream_t st)
{
    if (f16) {
        march::UpF16Slots<G> u16{(const uint16_t*)upl, eb_b};
        u16.stride = slot;
        return launch_level_group<G>(small_a, L, nx, nz, lop, u_stride,
                                     march::StoreF16EpiSlots<G>{(uint16_t*)outb, slot, eb_b}, dirs, u16, st);
    }
    march::UpF32 u32{(const float*)upl};
    u32.stride = slot;
    return launch_level_group<G>(small_a, L, nx, nz, lop, u_stride, march::StoreEpiSlots<G>{(float*)outb, slot},
                                 dirs, u32, st);
}

// Emergent intensity along a beam of parallel long characteristics (Sec.
// 3.9) through the synthesised fields: 4 rays x 16 wavelengths of one batch
// per wavefront, ray j from o0 + s_j p (s_j = j + 1/2 - n_rays/2) along d,
// the op's per-step opacity (the line op's Doppler shift follows d).
template <class Op>
__global__ __launch_bounds__(march::kBlock) void k_emergent_op(int32_t nx, int32_t nz, Op op, double ox0, double oz0,
                                                               double px, double pz, double4 d, int32_t n_rays,
                                                               float* __restrict__ out, int32_t lam0, int32_t n_valid)
{
    using march::kBlock;
    __shared__ uint4 seg[kBlock / 64][4][march::kSegRow];
    __shared__ typename Op::Stage stg[Op::kStaged ? kBlock / 64 : 1][4][march::kStgRow];
    __shared__ float2 op_smem[Op::kSmemBytes > 0 ? Op::kSmemBytes / 8 : 2];
    if constexpr (Op::kSmemBytes > 0) {
        op.init_shared(op_smem);
        __syncthreads();
    }
    const march::RowCtx c = march::row_ctx();
    op.init(c.l);
    seg[c.w][c.row][c.l] = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (Op::kStaged) {
        uint4* gw = reinterpret_cast<uint4*>(&stg[c.w][0][0]);
        constexpr int n16 = 4 * march::kStgRow * (int)sizeof(typename Op::Stage) / 16;
        for (int i = c.lane; i < n16; i += 64) gw[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    march::wave_sync();
    LevelDesc L{};
    L.ds_scale = 1.0;
    const int64_t stride = (int64_t)gridDim.x * march::kRaysPerBlock;
    for (int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + c.w) * 4; base < n_rays; base += stride) {
        const int64_t j = base + c.row;
        const bool active = j < n_rays;
        const double sj = (double)(active ? j : 0) + 0.5 - 0.5 * (double)n_rays;
        op.begin_ray(d.x, d.y);
        float I[1], T[1];
        march::walk_ray(L, nx, nz, op, ox0 + sj * px, oz0 + sj * pz, d, 0.0, INFINITY, active, seg[c.w],
                        stg[Op::kStaged ? c.w : 0], c, I, T);
        if (active && c.l < n_valid) out[(int64_t)(lam0 + c.l) * n_rays + j] = I[0];
    }
}

template <int NL>
hipError_t launch_se(rcx_nlte* s, const float* rates, double* pops, hipStream_t st)
{
    hipLaunchKernelGGL(k_stat_eq<NL>, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->atom, s->ncell, rates,
                       s->cup, s->cdn, s->ntot, pops, s->d_max, s->charge ? s->ne_copy : nullptr,
                       s->charge && s->pressure ? s->p_kt : nullptr, s->plan->mask_dev);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Batches b .. b + G - 1 march their cascades >= 1 together: the largest G
// in {4, 2} (at most gmax) whose batches all belong to batch b's line, else 1.
static int32_t line_group(const rcx_nlte* s, int32_t b, int32_t gmax)
{
    const int32_t nb = (int32_t)s->batches.size();
    if (s->atom.t[s->batches[b].trans].kind != 0) return 1;
    for (int32_t G = gmax; G >= 2; G /= 2) {
        bool same = b + G <= nb;
        for (int32_t k = 1; same && k < G; ++k) same = s->batches[b + k].trans == s->batches[b].trans;
        if (same) return G;
    }
    return 1;
}

int32_t rcx_nlte_create(const rcx_grid* g, const rcx_params* p, const rcx_atom* atom, int32_t n_wave,
                        const double* lambda_nm_host, const int32_t* trans_host, const double* dnu_host, rcx_nlte** out)
{
    if (out) *out = nullptr;
    if (!g || !p || !atom || !lambda_nm_host || !trans_host || !dnu_host || !out)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: null argument");
    if (n_wave <= 0) return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: n_wave must be positive");
    if (atom->n_levels < 2 || atom->n_levels > RCX_NLTE_MAX_LEVELS || atom->n_lines < 0 ||
        atom->n_lines > RCX_NLTE_MAX_LINES || atom->n_conts < 0 || atom->n_conts > RCX_NLTE_MAX_CONTS)
        return nlte_fail(RCX_E_UNSUPPORTED, "rcx_nlte_create: atom exceeds the supported sizes");
    if (p->c0_dirs != 4) return nlte_fail(RCX_E_UNSUPPORTED, "rcx_nlte_create: the rate epilogue needs c0_dirs = 4");
    if ((p->flags & ~RCX_FLAG_CHECK_INPUT) != 0)
        return nlte_fail(RCX_E_UNSUPPORTED, "rcx_nlte_create: only RCX_FLAG_CHECK_INPUT (basic merge only)");
    const int32_t nt = atom->n_lines + atom->n_conts;
    if (nt < 1) return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: no transitions");
    for (int32_t k = 0; k < atom->n_lines; ++k)
        if (atom->line_lower[k] < 0 || atom->line_upper[k] >= atom->n_levels ||
            atom->line_lower[k] >= atom->line_upper[k] || !(atom->line_lambda_nm[k] > 0) || !(atom->line_f[k] > 0))
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: bad line definition");
    for (int32_t k = 0; k < atom->n_conts; ++k)
        if (atom->cont_lower[k] < 0 || atom->cont_upper[k] != atom->n_levels - 1 || !(atom->cont_edge_nm[k] > 0))
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: bad continuum definition (upper must be the last level)");
    // wavelengths grouped by transition, in transition order
    for (int32_t l = 0; l < n_wave; ++l) {
        if (trans_host[l] < 0 || trans_host[l] >= nt)
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: transition index out of range");
        if (l > 0 && trans_host[l] < trans_host[l - 1])
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: wavelengths must be grouped by ascending transition");
        if (!(lambda_nm_host[l] > 0) || !(dnu_host[l] >= 0))
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: bad wavelength or weight");
        const int32_t t = trans_host[l];
        if (t >= atom->n_lines && lambda_nm_host[l] > atom->cont_edge_nm[t - atom->n_lines] * (1 + 1e-12))
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_create: continuum wavelength beyond its edge");
    }

    rcx_nlte* s = new (std::nothrow) rcx_nlte();
    if (!s) return nlte_fail(RCX_E_NOMEM, "rcx_nlte_create: host allocation");
    int32_t rc = rcx_plan_create(g, p, kLB, &s->plan);
    if (rc != RCX_OK) {
        delete s;
        return rc;
    }
    // the solver keeps its own field and cascade buffers: the plan's
    // workspace (sized for its inclination slots) is not needed
    if (s->plan->ws_own) {
        (void)hipFree(s->plan->ws_own);
        s->plan->ws_own = nullptr;
    }
    s->n_wave = n_wave;
    s->ncell = (int64_t)g->nx * g->nz;
    s->voxel = g->voxel_scale;
    s->lam_nm.assign(lambda_nm_host, lambda_nm_host + n_wave);
    s->dnu.assign(dnu_host, dnu_host + n_wave);
    s->trans.assign(trans_host, trans_host + n_wave);

    // atom in SI
    AtomDev& A = s->atom;
    A.nl = atom->n_levels;
    A.nt = nt;
    A.n_lines = atom->n_lines;
    A.n_conts = atom->n_conts;
    for (int l = 0; l < A.nl; ++l) {
        A.E[l] = atom->E_eV[l] * kQe;
        A.g[l] = atom->g[l];
    }
    A.mass = atom->mass_amu * kAmu;
    for (int k = 0; k < atom->n_lines; ++k) {
        Trans& t = A.t[k];
        t.kind = 0;
        t.i = atom->line_lower[k];
        t.j = atom->line_upper[k];
        t.line = k;
        t.nu0 = kC / (atom->line_lambda_nm[k] * 1e-9);
        t.sigma = kQe * kQe * atom->line_f[k] / (4.0 * kEps0 * kMe * kC);
        t.gr = A.g[t.i] / A.g[t.j];
        t.U0 = 2.0 * kH * t.nu0 * t.nu0 * t.nu0 / (kC * kC);
        t.q = atom->q_coll[k];
    }
    std::vector<double> Aein(atom->n_lines);
    for (int k = 0; k < atom->n_lines; ++k) {
        const Trans& t = A.t[k];
        Aein[k] = 2.0 * kPi * kQe * kQe * t.nu0 * t.nu0 * A.g[t.i] * atom->line_f[k] /
                  (kEps0 * kMe * kC * kC * kC * A.g[t.j]);
    }
    for (int k = 0; k < atom->n_lines; ++k) {  // natural damping: A out of the upper and the lower level
        double gsum = 0.0;
        for (int m = 0; m < atom->n_lines; ++m)
            if (A.t[m].j == A.t[k].j || A.t[m].j == A.t[k].i) gsum += Aein[m];
        A.t[k].gamma = gsum;
    }
    for (int k = 0; k < atom->n_conts; ++k) {
        Trans& t = A.t[atom->n_lines + k];
        t.kind = 1;
        t.i = atom->cont_lower[k];
        t.j = atom->cont_upper[k];
        t.line = k;
        t.nu0 = kC / (atom->cont_edge_nm[k] * 1e-9);
        t.sigma = atom->cont_alpha0[k];
        t.gr = A.g[t.i] / A.g[t.j];
        t.q = atom->q_coll[atom->n_lines + k];
    }

    // batches of <= 16 wavelengths within each transition's group
    s->tb0.assign(nt, 0);
    s->tb1.assign(nt, 0);
    int32_t l = 0;
    for (int32_t t = 0; t < nt; ++t) {
        s->tb0[t] = (int32_t)s->batches.size();
        while (l < n_wave && s->trans[l] == t) {
            int32_t n = 0;
            while (n < kLB && l + n < n_wave && s->trans[l + n] == t) ++n;
            const int32_t slot = A.t[t].kind == 1 ? s->n_cont_batches++ : -1;
            s->batches.push_back({t, l, n, slot});
            l += n;
        }
        s->tb1[t] = (int32_t)s->batches.size();
    }
    const int32_t nb = (int32_t)s->batches.size();
    std::vector<float> bc((size_t)nb * 5 * kLB, 0.0f);
    for (int32_t b = 0; b < nb; ++b) {
        const auto& B = s->batches[b];
        const Trans& t = A.t[B.trans];
        for (int32_t q = 0; q < B.n; ++q) {
            const int32_t lam = B.lam0 + q;
            const double nu = kC / (s->lam_nm[lam] * 1e-9);
            float* row = &bc[(size_t)b * 5 * kLB];
            row[0 * kLB + q] = (float)(4.0 * kPi * s->dnu[lam] / (kH * nu) / 4.0);
            if (t.kind == 0) {
                row[1 * kLB + q] = (float)(kC * (nu - t.nu0) / t.nu0);
            } else {
                row[2 * kLB + q] = (float)nu;
                row[3 * kLB + q] = (float)(t.sigma * std::pow(t.nu0 / nu, 3.0));
                row[4 * kLB + q] = (float)(2.0 * kH * nu * nu * nu / (kC * kC));
            }
        }
    }
    const int64_t nc = s->ncell;
    int64_t max_entries = 0;
    for (const auto& L : s->plan->levels) max_entries = std::max<int64_t>(max_entries, (int64_t)L.px * L.pz * L.nd);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    chk(dmalloc(s, &s->bconst, bc.size() * sizeof(float)));
    chk(dmalloc(s, &s->d_tb, sizeof(int32_t) * 2 * nt));
    chk(dmalloc(s, &s->lte, sizeof(double) * A.nl * nc));
    chk(dmalloc(s, &s->cup, sizeof(double) * nt * nc));
    chk(dmalloc(s, &s->cdn, sizeof(double) * nt * nc));
    chk(dmalloc(s, &s->T, sizeof(double) * nc));
    chk(dmalloc(s, &s->ntot, sizeof(double) * nc));
    chk(dmalloc(s, &s->ne_copy, sizeof(double) * nc));
    chk(dmalloc(s, &s->p_kt, sizeof(double) * nc));
    chk(dmalloc(s, &s->inv_vth, sizeof(float) * nc));
    chk(dmalloc(s, &s->adamp, sizeof(float) * std::max(1, A.n_lines) * nc));
    chk(dmalloc(s, &s->sphi, sizeof(float) * std::max(1, A.n_lines) * nc));
    chk(dmalloc(s, &s->lratio, sizeof(float) * std::max(1, A.n_conts) * nc));
    chk(dmalloc(s, &s->hkt2, sizeof(float) * nc));
    chk(dmalloc(s, &s->vel, sizeof(float2) * nc));
    chk(dmalloc(s, &s->line_rec, sizeof(float4) * std::max(1, A.n_lines) * nc));
    chk(dmalloc(s, &s->epi_rec, sizeof(float4) * nt * nc));
    chk(dmalloc(s, &s->Fcont, sizeof(float2) * std::max(1, s->n_cont_batches) * nc * kLB));
    // line groups need a slot per batch (and at least one cascade above 0)
    if (s->plan->n_casc >= 2 && !(s->plan->top_skipped && s->plan->n_casc == 2))
        for (int32_t b = 0; b < nb; ++b) s->group = std::max(s->group, line_group(s, b, 4));
    s->casc_slot = max_entries * kLB;
    chk(dmalloc(s, &s->casc[0], sizeof(float) * s->casc_slot * s->group));
    chk(dmalloc(s, &s->casc[1], sizeof(float) * s->casc_slot * s->group));
    chk(dmalloc(s, &s->part, sizeof(float2) * nb * nc));
    chk(dmalloc(s, &s->rates, sizeof(float) * 2 * nt * nc));
    chk(dmalloc(s, &s->d_max, sizeof(unsigned long long)));
    chk(dmalloc(s, &s->d_amax, sizeof(unsigned int)));
    chk(dmalloc(s, &s->d_check, sizeof(unsigned int)));
    chk(dmalloc(s, &s->vtab, sizeof(float2) * kNa * kNx));
    chk(dmalloc(s, &s->vtabc, sizeof(float2) * kNacMax * kNxc));
    chk(dmalloc(s, &s->u_all, sizeof(float) * n_wave));
    chk(dmalloc(s, &s->dnu_all, sizeof(float) * n_wave));
    chk(dmalloc(s, &s->norms, sizeof(float) * (12 + 2 * kMaxL)));
    s->f16 = p->storage == RCX_STORE_F16_SCALED;
    s->check_input = (p->flags & RCX_FLAG_CHECK_INPUT) != 0;
    chk(dmalloc(s, &s->smax, sizeof(unsigned int) * nb * kLB));
    chk(dmalloc(s, &s->ebias, sizeof(int32_t) * nb * kLB));
    if (e != hipSuccess) {
        rcx_nlte_destroy(s);
        return nlte_fail(RCX_E_NOMEM, std::string("rcx_nlte_create: hipMalloc: ") + hipGetErrorName(e));
    }
    std::vector<int32_t> tb(2 * nt);
    for (int t = 0; t < nt; ++t) {
        tb[t] = s->tb0[t];
        tb[nt + t] = s->tb1[t];
    }
    chk(hipMemcpy(s->bconst, bc.data(), bc.size() * sizeof(float), hipMemcpyHostToDevice));
    chk(hipMemcpy(s->d_tb, tb.data(), tb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    {
        std::vector<float> u(n_wave, 0.0f), d(n_wave);
        for (int32_t q = 0; q < n_wave; ++q) {
            const Trans& t = A.t[s->trans[q]];
            const double nu = kC / (s->lam_nm[q] * 1e-9);
            if (t.kind == 0) u[q] = (float)(kC * (nu - t.nu0) / t.nu0);
            d[q] = (float)s->dnu[q];
        }
        chk(hipMemcpy(s->u_all, u.data(), sizeof(float) * n_wave, hipMemcpyHostToDevice));
        chk(hipMemcpy(s->dnu_all, d.data(), sizeof(float) * n_wave, hipMemcpyHostToDevice));
    }
    if (e != hipSuccess) {
        rcx_nlte_destroy(s);
        return rcx::hip_fail(e, "rcx_nlte_create: hipMemcpy");
    }
    *out = s;
    return RCX_OK;
}

int32_t rcx_nlte_set_charge_conservation(rcx_nlte* s, int32_t enable)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_charge_conservation: null solver");
    s->charge = enable != 0;
    return RCX_OK;
}

int32_t rcx_nlte_set_temperature_cut(rcx_nlte* s, double t_cut, int64_t* level_active_host)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_temperature_cut: null solver");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_temperature_cut: set the atmosphere first");
    if (!(t_cut > 0.0)) return rcx_plan_set_active_host(s->plan, nullptr, level_active_host);
    std::vector<double> T((size_t)s->ncell);
    RCX_HIP_TRY(hipMemcpy(T.data(), s->T, sizeof(double) * s->ncell, hipMemcpyDeviceToHost));
    std::vector<uint8_t> flag((size_t)s->ncell);
    for (size_t c = 0; c < flag.size(); ++c) flag[c] = T[c] < t_cut ? 1 : 0;
    return rcx_plan_set_active_host(s->plan, flag.data(), level_active_host);
}

int32_t rcx_nlte_set_pressure_conservation(rcx_nlte* s, int32_t enable)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_pressure_conservation: null solver");
    if (enable && !s->charge)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_pressure_conservation: needs charge conservation");
    s->pressure = enable != 0;
    return RCX_OK;
}

static int32_t stat_eq(rcx_nlte* s, const float* rates, double* pops, double* change_host, hipStream_t st);

int32_t rcx_nlte_collisional_ne(rcx_nlte* s, int32_t n_iter, hipStream_t st)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_collisional_ne: null solver");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_collisional_ne: set the atmosphere first");
    if (n_iter < 1) return nlte_fail(RCX_E_INVALID, "rcx_nlte_collisional_ne: n_iter must be >= 1");
    // radiative rates zero; populations from LTE at the current n_e, then
    // equilibrium + charge steps on a temporary copy
    double* pops = nullptr;
    RCX_HIP_TRY(hipStreamSynchronize(st));
    RCX_HIP_TRY(hipMalloc((void**)&pops, sizeof(double) * s->atom.nl * s->ncell));
    const int64_t nr = (int64_t)s->atom.nt * 2 * s->ncell;
    hipLaunchKernelGGL(k_zero_u32n, dim3(blocks_for(nr, 256)), dim3(256), 0, st, (unsigned int*)s->rates,
                       (int32_t)nr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(pops, s->lte, sizeof(double) * s->atom.nl * s->ncell,
                                             hipMemcpyDeviceToDevice, st);
    const int32_t charge = s->charge, pressure = s->pressure;
    s->charge = 1;
    s->pressure = 0;
    int32_t rc = e == hipSuccess ? RCX_OK : rcx::hip_fail(e, "rcx_nlte_collisional_ne");
    for (int32_t it = 0; it < n_iter && rc == RCX_OK; ++it) {
        double ch = 0.0;
        rc = stat_eq(s, s->rates, pops, &ch, st);
    }
    s->charge = charge;
    s->pressure = pressure;
    const hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(pops);
    if (rc != RCX_OK) return rc;
    RCX_HIP_TRY(es);
    // the pressure held from here on is that of the atmosphere at this n_e
    hipLaunchKernelGGL(k_sum2, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->ncell, s->ntot, s->ne_copy,
                       s->p_kt);
    RCX_HIP_TRY(hipGetLastError());
    return RCX_OK;
}

int32_t rcx_nlte_get_ne(rcx_nlte* s, double* ne, hipStream_t st)
{
    if (!s || !ne) return nlte_fail(RCX_E_INVALID, "rcx_nlte_get_ne: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_get_ne: set the atmosphere first");
    RCX_HIP_TRY(hipMemcpyAsync(ne, s->ne_copy, sizeof(double) * s->ncell, hipMemcpyDeviceToDevice, st));
    return RCX_OK;
}

int32_t rcx_nlte_set_line_profile(rcx_nlte* s, int32_t mode)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_line_profile: null solver");
    if (mode != RCX_PROFILE_AUTO && mode != RCX_PROFILE_TABLE)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_line_profile: mode must be RCX_PROFILE_AUTO or RCX_PROFILE_TABLE");
    s->profile_mode = mode;
    return RCX_OK;
}

int32_t rcx_nlte_set_atmosphere(rcx_nlte* s, const double* T, const double* ne, const double* ntot, const float* vel,
                                hipStream_t st)
{
    if (!s || !T || !ne || !ntot || !vel) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_atmosphere: null argument");
    const int64_t nc = s->ncell;
    if (s->check_input) {
        // T, n_e, ntot finite and positive, velocities finite (synchronises)
        const double* pos[3] = {T, ne, ntot};
        const char* names[3] = {"rcx_nlte_set_atmosphere: T", "rcx_nlte_set_atmosphere: ne",
                                "rcx_nlte_set_atmosphere: ntot"};
        for (int q = 0; q < 3; ++q) {
            RCX_HIP_TRY(launch_zero_flag(s->d_check, st));
            RCX_HIP_TRY(launch_check_f64(pos[q], nc, kCheckPositive, s->d_check, st));
            const int32_t rc = check_flag_result(s->d_check, names[q], st);
            if (rc != RCX_OK) return rc;
        }
        RCX_HIP_TRY(launch_zero_flag(s->d_check, st));
        RCX_HIP_TRY(launch_check_f32(vel, 2 * nc, kCheckFinite, s->d_check, st));
        const int32_t rc = check_flag_result(s->d_check, "rcx_nlte_set_atmosphere: vel", st);
        if (rc != RCX_OK) return rc;
    }
    RCX_HIP_TRY(hipMemcpyAsync(s->T, T, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    RCX_HIP_TRY(hipMemcpyAsync(s->ntot, ntot, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    RCX_HIP_TRY(hipMemcpyAsync(s->ne_copy, ne, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_pack_vel, dim3(blocks_for(nc, 256)), dim3(256), 0, st, nc, vel, s->vel);
    RCX_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum2, dim3(blocks_for(nc, 256)), dim3(256), 0, st, nc, ntot, ne, s->p_kt);
    RCX_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, s->d_amax);
    RCX_HIP_TRY(hipGetLastError());
    StaticOut o{s->lte, s->cup, s->cdn, s->inv_vth, s->adamp, s->sphi, s->lratio, s->hkt2, s->d_amax};
    hipLaunchKernelGGL(k_static, dim3(blocks_for(nc, 256)), dim3(256), 0, st, s->atom, nc, s->T, ne, s->ntot, o);
    RCX_HIP_TRY(hipGetLastError());
    unsigned int bits = 0;
    RCX_HIP_TRY(hipMemcpyAsync(&bits, s->d_amax, sizeof(bits), hipMemcpyDeviceToHost, st));
    RCX_HIP_TRY(hipStreamSynchronize(st));
    float amax;
    std::memcpy(&amax, &bits, sizeof(amax));
    if (!(amax == amax)) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_atmosphere: damping is not finite (check T)");
    const double a_top = std::max(1.02 * (double)amax, 1e-8);
    const double da = a_top / (kNa - 1);
    s->v_inv_da = (float)(1.0 / da);
    hipLaunchKernelGGL(k_voigt_fill, dim3(blocks_for((int64_t)kNa * kNx, 128)), dim3(128), 0, st, s->vtab, da,
                       kXTab / (kNx - 1));
    RCX_HIP_TRY(hipGetLastError());
    s->small_a = s->profile_mode == RCX_PROFILE_AUTO && a_top <= kSmallAMax;
    if (s->small_a) {
        // the expansion in a: the g(x) = 1 - 2x F(x) table
        s->n_ac = 1;
        s->da_c = 1.0;
        hipLaunchKernelGGL(k_dawson_fill, dim3(blocks_for(kNg, 64)), dim3(64), 0, st, s->vtabc);
    } else {
        // compact table: a step of at most 2e-3 (linear-in-a error below
        // 1e-6), at most kNacMax nodes
        s->n_ac = (int32_t)std::min<double>(kNacMax, std::max(2.0, std::ceil(a_top / 2e-3) + 1.0));
        s->da_c = a_top / (s->n_ac - 1);
        hipLaunchKernelGGL(k_voigt_fill_compact, dim3(blocks_for((int64_t)s->n_ac * kNxc, 64)), dim3(64), 0, st,
                           s->vtabc, s->n_ac, s->da_c);
    }
    RCX_HIP_TRY(hipGetLastError());
    s->atm_set = true;
    return RCX_OK;
}

int32_t rcx_nlte_lte_populations(rcx_nlte* s, double* pops, hipStream_t st)
{
    if (!s || !pops) return nlte_fail(RCX_E_INVALID, "rcx_nlte_lte_populations: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_lte_populations: set the atmosphere first");
    RCX_HIP_TRY(hipMemcpyAsync(pops, s->lte, sizeof(double) * s->atom.nl * s->ncell, hipMemcpyDeviceToDevice, st));
    return RCX_OK;
}

static int32_t formal_solve_rates(rcx_nlte* s, const double* pops, float* rates, float* J, hipStream_t st)
{
    const rcx_plan* P = s->plan;
    const int32_t nx = P->grid.nx, nz = P->grid.nz;
    const int64_t nc = s->ncell;
    const AtomDev& A = s->atom;
    // record z: a itself for the expansion, a / da on the compact table
    SynthArgs sa{pops, s->inv_vth, s->adamp, s->sphi, s->lratio, s->hkt2, s->line_rec, s->epi_rec, s->voxel,
                 s->small_a ? 1.0f : (float)(1.0 / s->da_c), s->small_a ? (1 << 24) : s->n_ac};
    hipLaunchKernelGGL(k_synth, dim3(blocks_for(nc, 256)), dim3(256), 0, st, A, nc, sa);
    RCX_HIP_TRY(hipGetLastError());
    if (P->mask_dev && A.n_lines > 0) {
        // sparse (Sec. 3.5): unflagged cells transparent, no emission
        hipLaunchKernelGGL(k_mask_line_rec, dim3(blocks_for((int64_t)A.n_lines * nc, 256)), dim3(256), 0, st,
                           s->line_rec, P->mask_dev, nc, A.n_lines);
        RCX_HIP_TRY(hipGetLastError());
    }
    const int32_t nb = (int32_t)s->batches.size();
    if (s->f16) {
        hipLaunchKernelGGL(k_zero_u32n, dim3(blocks_for((int64_t)nb * kLB, 256)), dim3(256), 0, st, s->smax, nb * kLB);
        RCX_HIP_TRY(hipGetLastError());
    }
    // continuum fields (and the per-wavelength max S of every batch)
    for (int32_t b = 0; b < nb; ++b) {
        const auto& B = s->batches[b];
        const Trans& tr = A.t[B.trans];
        unsigned int* smax_b = s->f16 ? s->smax + (size_t)b * kLB : nullptr;
        if (tr.kind == 1) {
            ContBatch cb{};
            cb.trans = B.trans;
            cb.n = B.n;
            for (int q = 0; q < B.n; ++q) cb.nu[q] = kC / (s->lam_nm[B.lam0 + q] * 1e-9);
            float2* Fb = s->Fcont + (size_t)B.cont_slot * nc * kLB;
            hipLaunchKernelGGL(k_synth_cont, dim3(blocks_for(nc * kLB, 256)), dim3(256), 0, st, A, nc, pops, s->T, cb,
                               s->lratio, s->voxel, Fb, smax_b);
            RCX_HIP_TRY(hipGetLastError());
            if (P->mask_dev) RCX_HIP_TRY(launch_mask_fields(Fb, P->mask_dev, nc, 1, st));
        } else if (smax_b) {
            hipLaunchKernelGGL(k_smax_line, dim3(std::min<unsigned>(blocks_for(nc, 256), 1024u)), dim3(256), 0, st, nc,
                               s->line_rec + (size_t)tr.line * nc, smax_b);
            RCX_HIP_TRY(hipGetLastError());
        }
    }
    if (s->f16) RCX_HIP_TRY(launch_ebias(nb * kLB, s->smax, s->ebias, st));
    // 2D invariance (Sec. 3.1): every inclination m marches the flatland
    // rays with its path per projected cell 1/sin(theta_m) and sin(theta_m)
    // of the in-plane velocity; J and the rates sum w_m times its share
    for (int32_t m = 0; m < P->prm.n_incl; ++m) {
    const double path = P->incl_scale[m], wm = P->incl_w[m];
    for (int32_t b = 0; b < nb; ++b) {
        const auto& B = s->batches[b];
        const Trans& tr = A.t[B.trans];
        const float* bc = s->bconst + b * 5 * kLB;
        march::FieldOp fop{};
        fop.Fb = s->Fcont + (size_t)std::max(B.cont_slot, 0) * nc * kLB;
        fop.fb_bytes = (uint32_t)(nc * kLB * sizeof(float2));
        LineOp lop{};
        if (tr.kind == 0) {
            lop.rec = s->line_rec + (size_t)tr.line * nc;
            lop.vel = s->vel;
            lop.tabc = s->vtabc;
            lop.n_a = s->n_ac;
            lop.u_b = bc + 1 * kLB;
            lop.ncell = (uint32_t)nc;
            lop.da_sqrtpi = (float)(s->da_c / std::sqrt(kPi));
            lop.vscale = (float)(1.0 / path);
        }
        RatesEpi re{};
        re.part = s->part + b * nc;
        re.epi_rec = s->epi_rec + (size_t)B.trans * nc;
        re.W = bc;
        re.nu = bc + 2 * kLB;
        re.alpha = bc + 3 * kLB;
        re.U0c = bc + 4 * kLB;
        re.gr = (float)tr.gr;
        re.U0 = (float)tr.U0;
        re.ell_cells = (float)std::sqrt(0.5);
        re.voxel = (float)s->voxel;
        re.kind = tr.kind;
        re.path = (float)path;
        re.wgt = (float)wm;
        re.acc = m > 0;
        const int32_t* eb_b = s->ebias + (size_t)b * kLB;
        // this batch and the next G - 1 of the same line: cascades >= 1 in
        // one pass for all, cascade 0 per batch from its slot
        const int32_t G = s->group > 1 ? line_group(s, b, s->group) : 1;
        const int64_t slot = s->casc_slot;
        int cur = 0;
        const void* up = nullptr;
        for (int32_t i = P->n_casc - 1; i >= 0; --i) {
            if (P->top_skipped && i == P->n_casc - 1) continue;
            LevelDesc L = P->levels[i];
            L.ds_scale = path;
            // cascade 0 (the rate epilogue): the cell's own part of the
            // interval is added analytically by RatesEpi
            if (i == 0) L.ta = std::sqrt(0.5);
            const double4* dirs = P->dirs_dev + P->dir_off[i];
            float* outb = s->casc[cur];
            const void* upl = L.has_up ? up : nullptr;
            auto timed_begin = [&](rcx_nlte::Timed& tm, int32_t n_wl) -> int32_t {
                tm.steps = P->work.level_steps[i] / P->prm.n_incl * n_wl;
                RCX_HIP_TRY(hipEventCreate(&tm.a));
                hipError_t ee = hipEventCreate(&tm.b);
                if (ee != hipSuccess) {
                    (void)hipEventDestroy(tm.a);
                    return rcx::hip_fail(ee, "rcx_nlte timing");
                }
                (void)hipEventRecord(tm.a, st);
                return RCX_OK;
            };
            if (G > 1 && i == 0) {
                // cascade 0 of each batch of the group, reading its slot of
                // cascade 1 and writing its own slot of outb
                for (int32_t k = 0; k < G; ++k) {
                    const int32_t bk = b + k;
                    const auto& Bk = s->batches[bk];
                    const float* bck = s->bconst + bk * 5 * kLB;
                    const int32_t* eb_k = s->ebias + (size_t)bk * kLB;
                    LineOp lk = lop;
                    lk.u_b = bck + 1 * kLB;
                    RatesEpi rk = re;
                    rk.part = s->part + bk * nc;
                    rk.W = bck;
                    rk.nu = bck + 2 * kLB;
                    rk.alpha = bck + 3 * kLB;
                    rk.U0c = bck + 4 * kLB;
                    rk.out = outb + k * slot;
                    rcx_nlte::Timed tm{tr.kind, 0, nullptr, nullptr};
                    if (s->timing) {
                        const int32_t rt = timed_begin(tm, Bk.n);
                        if (rt != RCX_OK) return rt;
                    }
                    hipError_t e;
                    if (s->f16) {
                        const march::UpF16 u16{upl ? (const uint16_t*)upl + k * slot : nullptr, eb_k};
                        e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lk, fop, rk, dirs, u16, st);
                    } else {
                        const march::UpF32 u32{upl ? (const float*)upl + k * slot : nullptr};
                        e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lk, fop, rk, dirs, u32, st);
                    }
                    if (s->timing) {
                        (void)hipEventRecord(tm.b, st);
                        s->pending.push_back(tm);
                    }
                    RCX_HIP_TRY(e);
                    if (J) RCX_HIP_TRY(launch_j(outb + k * slot, J, Bk.lam0, Bk.n, nc, 4, (float)wm, m > 0, st));
                }
                up = nullptr;
                break;
            }
            rcx_nlte::Timed tm{tr.kind, 0, nullptr, nullptr};
            if (s->timing) {
                int32_t n_wl = 0;
                for (int32_t k = 0; k < G; ++k) n_wl += s->batches[b + k].n;
                const int32_t rt = timed_begin(tm, n_wl);
                if (rt != RCX_OK) return rt;
            }
            hipError_t e;
            if (G == 4) {
                // cascades >= 1 of the 4 batches (slot w: batch b + w)
                e = launch_group_casc<4>(s->f16, s->small_a, L, nx, nz, lop, 5 * kLB, outb, upl, slot, eb_b, dirs, st);
            } else if (G == 2) {
                e = launch_group_casc<2>(s->f16, s->small_a, L, nx, nz, lop, 5 * kLB, outb, upl, slot, eb_b, dirs, st);
            } else if (s->f16) {
                // cascades >= 1 stored in FP16; cascade 0 (rates, J) in FP32
                const march::UpF16 u16{(const uint16_t*)upl, eb_b};
                if (i > 0) {
                    e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lop, fop, march::StoreF16Epi{(uint16_t*)outb, eb_b},
                                        dirs, u16, st);
                } else {
                    re.out = outb;
                    e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lop, fop, re, dirs, u16, st);
                }
            } else {
                const march::UpF32 u32{(const float*)upl};
                if (i > 0) {
                    e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lop, fop, march::StoreEpi{outb}, dirs, u32, st);
                } else {
                    re.out = outb;
                    e = launch_level_op(tr.kind, s->small_a, L, nx, nz, lop, fop, re, dirs, u32, st);
                }
            }
            if (s->timing) {
                (void)hipEventRecord(tm.b, st);
                s->pending.push_back(tm);
            }
            RCX_HIP_TRY(e);
            up = outb;
            cur ^= 1;
        }
        if (G > 1) {
            b += G - 1;  // the group's batches were marched with this one (and their J written)
            continue;
        }
        if (J) RCX_HIP_TRY(launch_j((const float*)up, J, B.lam0, B.n, nc, 4, (float)wm, m > 0, st));
    }
    }
    hipLaunchKernelGGL(k_rates_sum, dim3(blocks_for(nc, 256)), dim3(256), 0, st, nc, A.nt, s->d_tb, s->d_tb + A.nt,
                       s->part, rates);
    RCX_HIP_TRY(hipGetLastError());
    if (P->mask_dev) {
        // sparse: no rays reach the unflagged cells' partial sums; their
        // rates and J are 0
        RCX_HIP_TRY(launch_mask_j(rates, P->mask_dev, nc, 2 * A.nt, st));
        if (J) RCX_HIP_TRY(launch_mask_j(J, P->mask_dev, nc, s->n_wave, st));
    }
    return RCX_OK;
}

int32_t rcx_nlte_emergent(rcx_nlte* s, const double* pops, double wx, double wz, int32_t n_rays, float* I,
                          hipStream_t st)
{
    if (!s || !pops || !I) return nlte_fail(RCX_E_INVALID, "rcx_nlte_emergent: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_emergent: set the atmosphere first");
    if (n_rays <= 0) return nlte_fail(RCX_E_INVALID, "rcx_nlte_emergent: n_rays must be positive");
    const double wn = std::hypot(wx, wz);
    if (!(wn > 0.0) || !std::isfinite(wn)) return nlte_fail(RCX_E_INVALID, "rcx_nlte_emergent: zero direction");
    wx /= wn;
    wz /= wn;
    const rcx_plan* P = s->plan;
    const int32_t nx = P->grid.nx, nz = P->grid.nz;
    const int64_t nc = s->ncell;
    const AtomDev& A = s->atom;
    // the fields of the populations, as for the formal solve
    SynthArgs sa{pops, s->inv_vth, s->adamp, s->sphi, s->lratio, s->hkt2, s->line_rec, s->epi_rec, s->voxel,
                 s->small_a ? 1.0f : (float)(1.0 / s->da_c), s->small_a ? (1 << 24) : s->n_ac};
    hipLaunchKernelGGL(k_synth, dim3(blocks_for(nc, 256)), dim3(256), 0, st, A, nc, sa);
    RCX_HIP_TRY(hipGetLastError());
    if (P->mask_dev && A.n_lines > 0) {
        hipLaunchKernelGGL(k_mask_line_rec, dim3(blocks_for((int64_t)A.n_lines * nc, 256)), dim3(256), 0, st,
                           s->line_rec, P->mask_dev, nc, A.n_lines);
        RCX_HIP_TRY(hipGetLastError());
    }
    const int32_t nb = (int32_t)s->batches.size();
    for (int32_t b = 0; b < nb; ++b) {
        const auto& B = s->batches[b];
        const Trans& tr = A.t[B.trans];
        if (tr.kind != 1) continue;
        ContBatch cb{};
        cb.trans = B.trans;
        cb.n = B.n;
        for (int q = 0; q < B.n; ++q) cb.nu[q] = kC / (s->lam_nm[B.lam0 + q] * 1e-9);
        float2* Fb = s->Fcont + (size_t)B.cont_slot * nc * kLB;
        hipLaunchKernelGGL(k_synth_cont, dim3(blocks_for(nc * kLB, 256)), dim3(256), 0, st, A, nc, pops, s->T, cb,
                           s->lratio, s->voxel, Fb, nullptr);
        RCX_HIP_TRY(hipGetLastError());
        if (P->mask_dev) RCX_HIP_TRY(launch_mask_fields(Fb, P->mask_dev, nc, 1, st));
    }
    // the beam (as rcx_emergent): from outside the domain on the observer's
    // side, march direction -w
    const double R = 0.5 * std::hypot((double)nx, (double)nz) + 2.0;
    const double ox0 = 0.5 * nx + R * wx, oz0 = 0.5 * nz + R * wz;
    double dx = -wx, dz = -wz;
    if (std::fabs(dx) < 1e-12) dx = dx < 0.0 ? -1e-12 : 1e-12;
    if (std::fabs(dz) < 1e-12) dz = dz < 0.0 ? -1e-12 : 1e-12;
    const double4 d = make_double4(dx, dz, 1.0 / dx, 1.0 / dz);
    const dim3 grid = march_grid(n_rays);
    for (int32_t b = 0; b < nb; ++b) {
        const auto& B = s->batches[b];
        const Trans& tr = A.t[B.trans];
        const float* bc = s->bconst + b * 5 * kLB;
        if (tr.kind == 1) {
            march::FieldOp fop{};
            fop.Fb = s->Fcont + (size_t)B.cont_slot * nc * kLB;
            fop.fb_bytes = (uint32_t)(nc * kLB * sizeof(float2));
            hipLaunchKernelGGL(k_emergent_op<march::FieldOp>, grid, dim3(march::kBlock), 0, st, nx, nz, fop, ox0, oz0,
                               -wz, wx, d, n_rays, I, B.lam0, B.n);
        } else if (s->small_a) {
            LineOpSmallA sop{};
            sop.rec = s->line_rec + (size_t)tr.line * nc;
            sop.vel = s->vel;
            sop.tabc = s->vtabc;
            sop.n_a = s->n_ac;
            sop.u_b = bc + 1 * kLB;
            sop.ncell = (uint32_t)nc;
            sop.da_sqrtpi = (float)(s->da_c / std::sqrt(kPi));
            hipLaunchKernelGGL(k_emergent_op<LineOpSmallA>, grid, dim3(march::kBlock), 0, st, nx, nz, sop, ox0, oz0,
                               -wz, wx, d, n_rays, I, B.lam0, B.n);
        } else {
            LineOp lop{};
            lop.rec = s->line_rec + (size_t)tr.line * nc;
            lop.vel = s->vel;
            lop.tabc = s->vtabc;
            lop.n_a = s->n_ac;
            lop.u_b = bc + 1 * kLB;
            lop.ncell = (uint32_t)nc;
            lop.da_sqrtpi = (float)(s->da_c / std::sqrt(kPi));
            hipLaunchKernelGGL(k_emergent_op<LineOp>, grid, dim3(march::kBlock), 0, st, nx, nz, lop, ox0, oz0, -wz,
                               wx, d, n_rays, I, B.lam0, B.n);
        }
        RCX_HIP_TRY(hipGetLastError());
    }
    return RCX_OK;
}

int32_t rcx_nlte_formal_solve_rates(rcx_nlte* s, const double* pops, float* rates, float* J, hipStream_t st)
{
    if (!s || !pops || !rates) return nlte_fail(RCX_E_INVALID, "rcx_nlte_formal_solve_rates: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_formal_solve_rates: set the atmosphere first");
    return formal_solve_rates(s, pops, rates, J, st);
}

// ---------------------------------------------------- Ng acceleration
// Ng (1974), in the least-squares form of Auer (1987): with iterates x_0
// (newest) .. x_{M+1} and differences d_k = x_k - x_{k+1}, choose c_1..c_M
// minimising sum w (d_0 - sum_j c_j (d_0 - d_j))^2 with w = 1 / x_0^2, i.e.
// A c = b, A_ij = sum w (d_0 - d_i)(d_0 - d_j), b_i = sum w d_0 (d_0 - d_i);
// then x = (1 - sum_j c_j) x_0 + sum_j c_j x_j.
constexpr int kNgMaxOrder = 3;
constexpr int kNgSums = kNgMaxOrder * (kNgMaxOrder + 1) / 2 + kNgMaxOrder;
constexpr int kNgBlocks = 512;

struct NgPtrs {
    const double* x[kNgMaxOrder + 2];  // x_0 newest
};

__global__ __launch_bounds__(256) void k_ng_sums(NgPtrs P, int32_t M, int64_t n, double* __restrict__ part)
{
    double acc[kNgSums];
#pragma unroll
    for (int k = 0; k < kNgSums; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x[kNgMaxOrder + 2], d[kNgMaxOrder + 1];
        for (int k = 0; k < M + 2; ++k) x[k] = P.x[k][i];
        for (int k = 0; k < M + 1; ++k) d[k] = x[k] - x[k + 1];
        const double w = 1.0 / (x[0] * x[0]);
        int q = 0;
        for (int a = 1; a <= M; ++a)
            for (int b = a; b <= M; ++b) acc[q++] += w * (d[0] - d[a]) * (d[0] - d[b]);
        for (int a = 1; a <= M; ++a) acc[q++] += w * d[0] * (d[0] - d[a]);
    }
    // block sum in a fixed order (deterministic)
    __shared__ double red[kNgSums][256];
    for (int k = 0; k < kNgSums; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < kNgSums; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kNgSums) part[(int64_t)blockIdx.x * kNgSums + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_ng_reduce(const double* __restrict__ part, int32_t nblocks, double* __restrict__ sums)
{
    if (threadIdx.x < kNgSums) {
        double t = 0.0;
        for (int b = 0; b < nblocks; ++b) t += part[(int64_t)b * kNgSums + threadIdx.x];
        sums[threadIdx.x] = t;
    }
}

struct NgCoef {
    double c[kNgMaxOrder];
};

__global__ void k_ng_update(NgPtrs P, int32_t M, NgCoef C, int64_t n, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double csum = 0.0, v = 0.0;
    for (int j = 1; j <= M; ++j) {
        csum += C.c[j - 1];
        v += C.c[j - 1] * P.x[j][i];
    }
    out[i] = (1.0 - csum) * P.x[0][i] + v;
}

// Solve the M x M system (partial pivoting); false if it is singular.
static bool ng_solve(int M, double A[kNgMaxOrder][kNgMaxOrder], double b[kNgMaxOrder], double c[kNgMaxOrder])
{
    for (int k = 0; k < M; ++k) {
        int piv = k;
        for (int r = k + 1; r < M; ++r)
            if (std::fabs(A[r][k]) > std::fabs(A[piv][k])) piv = r;
        if (!(std::fabs(A[piv][k]) > 0.0)) return false;
        if (piv != k) {
            for (int cc = 0; cc < M; ++cc) std::swap(A[k][cc], A[piv][cc]);
            std::swap(b[k], b[piv]);
        }
        for (int r = k + 1; r < M; ++r) {
            const double f = A[r][k] / A[k][k];
            for (int cc = k; cc < M; ++cc) A[r][cc] -= f * A[k][cc];
            b[r] -= f * b[k];
        }
    }
    for (int k = M - 1; k >= 0; --k) {
        double t = b[k];
        for (int cc = k + 1; cc < M; ++cc) t -= A[k][cc] * c[cc];
        c[k] = t / A[k][k];
        if (!std::isfinite(c[k])) return false;
    }
    return true;
}

// After an iteration: keep pops in the ring; when the schedule says so and
// M + 2 iterates are held, replace pops by the extrapolation (the ring then
// restarts from it).
static int32_t ng_step(rcx_nlte* s, double* pops, hipStream_t st)
{
    const int32_t M = s->ng_order;
    const int64_t n = (int64_t)s->atom.nl * s->ncell;
    const int32_t slots = M + 2;
    ++s->ng_iter;
    RCX_HIP_TRY(hipMemcpyAsync(s->ng_hist + (size_t)s->ng_head * n, pops, sizeof(double) * n,
                               hipMemcpyDeviceToDevice, st));
    s->ng_head = (s->ng_head + 1) % slots;
    s->ng_count = std::min(s->ng_count + 1, slots);
    if (s->ng_count < slots || s->ng_iter < s->ng_delay || (s->ng_iter - s->ng_delay) % s->ng_period != 0)
        return RCX_OK;
    NgPtrs P{};
    for (int k = 0; k < slots; ++k)  // newest first
        P.x[k] = s->ng_hist + (size_t)((s->ng_head - 1 - k + 2 * slots) % slots) * n;
    hipLaunchKernelGGL(k_ng_sums, dim3(kNgBlocks), dim3(256), 0, st, P, M, n, s->ng_part);
    RCX_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ng_reduce, dim3(1), dim3(64), 0, st, s->ng_part, kNgBlocks, s->ng_sums);
    RCX_HIP_TRY(hipGetLastError());
    double sums[kNgSums];
    RCX_HIP_TRY(hipMemcpyAsync(sums, s->ng_sums, sizeof(sums), hipMemcpyDeviceToHost, st));
    RCX_HIP_TRY(hipStreamSynchronize(st));
    double A[kNgMaxOrder][kNgMaxOrder], b[kNgMaxOrder], c[kNgMaxOrder];
    int q = 0;
    for (int a = 0; a < M; ++a)
        for (int bb = a; bb < M; ++bb) A[a][bb] = A[bb][a] = sums[q++];
    for (int a = 0; a < M; ++a) b[a] = sums[q++];
    if (!ng_solve(M, A, b, c)) return RCX_OK;  // degenerate: keep the plain iterate
    NgCoef C{};
    for (int j = 0; j < M; ++j) C.c[j] = c[j];
    hipLaunchKernelGGL(k_ng_update, dim3(blocks_for(n, 256)), dim3(256), 0, st, P, M, C, n, pops);
    RCX_HIP_TRY(hipGetLastError());
    // restart the ring from the extrapolated iterate
    RCX_HIP_TRY(hipMemcpyAsync(s->ng_hist, pops, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    s->ng_head = 1 % slots;
    s->ng_count = 1;
    return RCX_OK;
}

int32_t rcx_nlte_set_acceleration(rcx_nlte* s, int32_t order, int32_t delay, int32_t period)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_acceleration: null solver");
    if (order < 0 || order > kNgMaxOrder || delay < 0 || period < 1)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_acceleration: order in [0, 3], delay >= 0, period >= 1");
    const int64_t n = (int64_t)s->atom.nl * s->ncell;
    if (order > 0 && !s->ng_hist) {
        if (dmalloc(s, &s->ng_hist, sizeof(double) * (kNgMaxOrder + 2) * n) != hipSuccess ||
            dmalloc(s, &s->ng_part, sizeof(double) * kNgBlocks * kNgSums) != hipSuccess ||
            dmalloc(s, &s->ng_sums, sizeof(double) * kNgSums) != hipSuccess)
            return nlte_fail(RCX_E_NOMEM, "rcx_nlte_set_acceleration: device allocation");
    }
    s->ng_order = order;
    s->ng_delay = delay;
    s->ng_period = period;
    s->ng_count = s->ng_head = s->ng_iter = 0;
    return RCX_OK;
}

static int32_t stat_eq(rcx_nlte* s, const float* rates, double* pops, double* change_host, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, s->d_max);
    RCX_HIP_TRY(hipGetLastError());
    hipError_t e = hipErrorInvalidValue;
    switch (s->atom.nl) {
    case 2: e = launch_se<2>(s, rates, pops, st); break;
    case 3: e = launch_se<3>(s, rates, pops, st); break;
    case 4: e = launch_se<4>(s, rates, pops, st); break;
    case 5: e = launch_se<5>(s, rates, pops, st); break;
    case 6: e = launch_se<6>(s, rates, pops, st); break;
    default: return nlte_fail(RCX_E_UNSUPPORTED, "stat_eq: level count");
    }
    RCX_HIP_TRY(e);
    if (s->charge) {
        // LTE populations, collisional rates and continuum LTE ratios at the
        // new n_e (the damping maximum does not depend on n_e)
        StaticOut o{s->lte, s->cup, s->cdn, s->inv_vth, s->adamp, s->sphi, s->lratio, s->hkt2, s->d_amax};
        hipLaunchKernelGGL(k_static, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->atom, s->ncell, s->T,
                           s->ne_copy, s->ntot, o);
        RCX_HIP_TRY(hipGetLastError());
    }
    unsigned long long bits = 0;
    RCX_HIP_TRY(hipMemcpyAsync(&bits, s->d_max, sizeof(bits), hipMemcpyDeviceToHost, st));
    RCX_HIP_TRY(hipStreamSynchronize(st));
    double ch;
    std::memcpy(&ch, &bits, sizeof(ch));
    *change_host = ch;
    return RCX_OK;
}

int32_t rcx_nlte_stat_eq(rcx_nlte* s, const float* rates, double* pops, double* change_host, hipStream_t st)
{
    if (!s || !rates || !pops || !change_host) return nlte_fail(RCX_E_INVALID, "rcx_nlte_stat_eq: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_stat_eq: set the atmosphere first");
    return stat_eq(s, rates, pops, change_host, st);
}

int32_t rcx_nlte_iterate(rcx_nlte* s, double* pops, int32_t max_iter, double tol, int32_t* iters_host,
                         double* last_change_host, hipStream_t st)
{
    if (!s || !pops || !iters_host || !last_change_host)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_iterate: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_iterate: set the atmosphere first");
    if (max_iter < 1) return nlte_fail(RCX_E_INVALID, "rcx_nlte_iterate: max_iter must be >= 1");
    *iters_host = 0;
    *last_change_host = INFINITY;
    for (int32_t it = 0; it < max_iter; ++it) {
        int32_t rc = formal_solve_rates(s, pops, s->rates, nullptr, st);
        if (rc != RCX_OK) return rc;
        double ch = 0.0;
        rc = stat_eq(s, s->rates, pops, &ch, st);
        if (rc != RCX_OK) return rc;
        *iters_host = it + 1;
        *last_change_host = ch;
        if (ch < tol) return RCX_OK;
        if (s->ng_order > 0) {
            rc = ng_step(s, pops, st);
            if (rc != RCX_OK) return rc;
        }
    }
    return RCX_W_NOT_CONVERGED;
}

int32_t rcx_nlte_voigt_eval(rcx_nlte* s, int32_t n, const float* a, const float* x, float* out, hipStream_t st)
{
    if (!s || !a || !x || !out || n < 0) return nlte_fail(RCX_E_INVALID, "rcx_nlte_voigt_eval: bad argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_voigt_eval: set the atmosphere first");
    if (n == 0) return RCX_OK;
    const VoigtTab vt{s->vtab, s->v_inv_da, (float)((kNx - 1) / kXTab)};
    hipLaunchKernelGGL(k_voigt_eval, dim3(blocks_for(n, 256)), dim3(256), 0, st, vt, n, a, x, out);
    RCX_HIP_TRY(hipGetLastError());
    return RCX_OK;
}

int32_t rcx_nlte_voigt_eval_march(rcx_nlte* s, int32_t n, const float* a, const float* x, float* out, hipStream_t st)
{
    if (!s || !a || !x || !out || n < 0) return nlte_fail(RCX_E_INVALID, "rcx_nlte_voigt_eval_march: bad argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_voigt_eval_march: set the atmosphere first");
    if (n == 0) return RCX_OK;
    hipLaunchKernelGGL(k_voigt_eval_compact, dim3(blocks_for(n, 256)), dim3(256), 0, st, s->vtabc, s->n_ac,
                       (float)(1.0 / s->da_c), (float)(s->da_c / std::sqrt(kPi)), (int32_t)s->small_a, n, a, x, out);
    RCX_HIP_TRY(hipGetLastError());
    return RCX_OK;
}

int32_t rcx_nlte_dims(const rcx_nlte* s, int32_t* nl, int32_t* nt)
{
    if (!s || !nl || !nt) return nlte_fail(RCX_E_INVALID, "rcx_nlte_dims: null argument");
    *nl = s->atom.nl;
    *nt = s->atom.nt;
    return RCX_OK;
}

int32_t rcx_nlte_autotune(rcx_nlte* s, const char* cache_path, hipStream_t stream)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_autotune: null solver");
    // the solver marches with its plan's launch orders (results do not
    // depend on them): tune them on the plan's own formal solve
    return rcx_autotune(s->plan, cache_path, stream);
}

int32_t rcx_nlte_set_timing(rcx_nlte* s, int32_t enable)
{
    if (!s) return nlte_fail(RCX_E_INVALID, "rcx_nlte_set_timing: null solver");
    if (enable) {
        rcx_work w;  // per-cascade step counts for the records
        const int32_t rc = rcx_plan_work(s->plan, &w);
        if (rc != RCX_OK) return rc;
    }
    s->timing = enable != 0;
    return RCX_OK;
}

int32_t rcx_nlte_get_timing(rcx_nlte* s, double* ms_host, int64_t* launches_host, int64_t* steps_host)
{
    if (!s || !ms_host || !launches_host || !steps_host)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_get_timing: null argument");
    for (int k = 0; k < 2; ++k) {
        ms_host[k] = 0.0;
        launches_host[k] = 0;
        steps_host[k] = 0;
    }
    int32_t rc = RCX_OK;
    for (auto& t : s->pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && rc == RCX_OK) rc = rcx::hip_fail(e, "rcx_nlte_get_timing");
        const int k = t.kind == 0 ? 0 : 1;
        ms_host[k] += ms;
        ++launches_host[k];
        steps_host[k] += t.steps;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    s->pending.clear();
    return rc;
}

int32_t rcx_nlte_destroy(rcx_nlte* s)
{
    if (!s) return RCX_OK;
    for (auto& t : s->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->plan) rcx_plan_destroy(s->plan);
    delete s;
    return RCX_OK;
}

}  // extern "C"

static int32_t ensure_warm_buffers(rcx_nlte* s)
{
    if (s->Jtmp) return RCX_OK;
    if (dmalloc(s, &s->Jtmp, sizeof(float) * s->n_wave * s->ncell) != hipSuccess ||
        dmalloc(s, &s->feat, sizeof(float) * 6 * s->ncell) != hipSuccess ||
        dmalloc(s, &s->pred, sizeof(float) * kMaxL * s->ncell) != hipSuccess)
        return nlte_fail(RCX_E_NOMEM, "warm start buffers");
    return RCX_OK;
}

static int32_t features(rcx_nlte* s, const float* J, const float* norm_host, float* out, hipStream_t st)
{
    std::vector<float> nrm(12);
    for (int q = 0; q < 12; ++q) nrm[q] = norm_host ? norm_host[q] : (q < 6 ? 0.0f : 1.0f);
    RCX_HIP_TRY(hipMemcpyAsync(s->norms, nrm.data(), sizeof(float) * 12, hipMemcpyHostToDevice, st));
    FeatArgs f{};
    f.J = J;
    f.T = s->T;
    f.ne = s->ne_copy;
    f.vel = s->vel;
    f.inv_vth = s->inv_vth;
    f.adamp = s->adamp;
    f.line_rec = s->line_rec;
    f.u_all = s->u_all;
    f.dnu_all = s->dnu_all;
    f.n_lines = s->atom.n_lines;
    for (int t = 0; t < 2; ++t) {
        f.lam0[t] = f.lam1[t] = 0;
        if (t < s->atom.n_lines) {
            f.lam0[t] = s->batches[s->tb0[t]].lam0;
            const auto& last = s->batches[s->tb1[t] - 1];
            f.lam1[t] = last.lam0 + last.n;
        }
    }
    f.voxel = (float)s->voxel;
    f.norm = s->norms;
    f.out = out;
    const VoigtTab vt{s->vtab, s->v_inv_da, (float)((kNx - 1) / kXTab)};
    hipLaunchKernelGGL(k_features, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->ncell, vt, f);
    RCX_HIP_TRY(hipGetLastError());
    // norms must not be overwritten before the kernel has read them
    RCX_HIP_TRY(hipStreamSynchronize(st));
    return RCX_OK;
}

extern "C" {

int32_t rcx_nlte_features(rcx_nlte* s, const double* pops, const float* norm_host, float* feat, hipStream_t st)
{
    if (!s || !pops || !feat) return nlte_fail(RCX_E_INVALID, "rcx_nlte_features: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_features: set the atmosphere first");
    int32_t rc = ensure_warm_buffers(s);
    if (rc != RCX_OK) return rc;
    rc = formal_solve_rates(s, pops, s->rates, s->Jtmp, st);
    if (rc != RCX_OK) return rc;
    return features(s, s->Jtmp, norm_host, feat, st);
}

int32_t rcx_nlte_log_departures(rcx_nlte* s, const double* pops, const float* norm_host, float* out, hipStream_t st)
{
    if (!s || !pops || !out) return nlte_fail(RCX_E_INVALID, "rcx_nlte_log_departures: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_log_departures: set the atmosphere first");
    const int nl = s->atom.nl;
    std::vector<float> nrm(2 * nl);
    for (int q = 0; q < 2 * nl; ++q) nrm[q] = norm_host ? norm_host[q] : (q < nl ? 0.0f : 1.0f);
    RCX_HIP_TRY(hipMemcpyAsync(s->norms + 12, nrm.data(), sizeof(float) * 2 * nl, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_log_departures, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->ncell, nl, pops, s->lte,
                       s->norms + 12, out);
    RCX_HIP_TRY(hipGetLastError());
    RCX_HIP_TRY(hipStreamSynchronize(st));
    return RCX_OK;
}

// Populations from standardised predicted targets y [ncell][n_levels] on
// the stream (norms copied to the solver's device buffer first).
static int32_t pops_from_prediction(rcx_nlte* s, const float* y, const float* targ_norm_host, double* pops_out,
                                    hipStream_t st)
{
    const int nl = s->atom.nl;
    RCX_HIP_TRY(hipMemcpyAsync(s->norms + 12, targ_norm_host, sizeof(float) * 2 * nl, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_pops_from_pred, dim3(blocks_for(s->ncell, 256)), dim3(256), 0, st, s->ncell, nl, y,
                       s->norms + 12, s->lte, s->ntot, pops_out);
    RCX_HIP_TRY(hipGetLastError());
    // the norms buffer must not be overwritten before the kernel has read it
    RCX_HIP_TRY(hipStreamSynchronize(st));
    return RCX_OK;
}

int32_t rcx_nlte_pops_from_prediction(rcx_nlte* s, const float* y, const float* targ_norm_host, double* pops_out,
                                      hipStream_t st)
{
    if (!s || !y || !targ_norm_host || !pops_out)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_pops_from_prediction: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_pops_from_prediction: set the atmosphere first");
    const int nl = s->atom.nl;
    for (int q = nl; q < 2 * nl; ++q)
        if (!(targ_norm_host[q] > 0.0f) || !std::isfinite(targ_norm_host[q]) || !std::isfinite(targ_norm_host[q - nl]))
            return nlte_fail(RCX_E_INVALID, "rcx_nlte_pops_from_prediction: norms must be finite, stds positive");
    return pops_from_prediction(s, y, targ_norm_host, pops_out, st);
}

int32_t rcx_nlte_warm_start(rcx_nlte* s, rcx_mlp* net, const float* feat_norm_host, const float* targ_norm_host,
                            double* pops_out, hipStream_t st)
{
    if (!s || !net || !feat_norm_host || !targ_norm_host || !pops_out)
        return nlte_fail(RCX_E_INVALID, "rcx_nlte_warm_start: null argument");
    if (!s->atm_set) return nlte_fail(RCX_E_INVALID, "rcx_nlte_warm_start: set the atmosphere first");
    int32_t rc = ensure_warm_buffers(s);
    if (rc != RCX_OK) return rc;
    const int nl = s->atom.nl;
    RCX_HIP_TRY(hipMemcpyAsync(pops_out, s->lte, sizeof(double) * nl * s->ncell, hipMemcpyDeviceToDevice, st));
    rc = formal_solve_rates(s, pops_out, s->rates, s->Jtmp, st);
    if (rc != RCX_OK) return rc;
    rc = features(s, s->Jtmp, feat_norm_host, s->feat, st);
    if (rc != RCX_OK) return rc;
    rc = rcx_mlp_forward(net, s->feat, s->pred, (int32_t)s->ncell, st);
    if (rc != RCX_OK) return rc;
    return pops_from_prediction(s, s->pred, targ_norm_host, pops_out, st);
}

}  // extern "C"
