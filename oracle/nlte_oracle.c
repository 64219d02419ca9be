/*
 * nlte_oracle.c -- FP64 CPU oracle pieces of the non-LTE iteration of
 * Osborne & Sannikov (arXiv:2408.14425, Sec. 3.3) that need the cascade
 * solver: the Voigt function and the direction-dependent opacity of
 * Doppler-shifted lines seen by every ray step (Sec. 3.2: velocity-dependent
 * terms evaluated per ray, in the observer's frame).
 *
 * TEST INFRASTRUCTURE ONLY (see rc_oracle.c). Shares nothing with the HIP
 * library.
 *
 * Voigt function: H(a, x) = Re w(x + i a), w the Faddeeva function, computed
 * with J.A.C. Weideman's rational series ("Computation of the complex error
 * function", SIAM J. Numer. Anal. 31 (1994) 1497-1518): with L = sqrt(N /
 * sqrt 2) and Z = (L + i z)/(L - i z),
 *   w(z) = 2 p(Z) / (L - i z)^2 + pi^{-1/2} / (L - i z),  p(Z) = sum_{n=1..N} a_n Z^{n-1},
 * where a_n are the Fourier coefficients of (L^2 + t^2) e^{-t^2} sampled at
 * t = L tan(theta/2). Valid for Im z > 0. N = 40 here.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "rc_oracle.h"

#define WEI_N 40

static double wei_a[WEI_N + 1]; /* a_1 .. a_N */
static double wei_L;
static int wei_ready = 0;

static void wei_init(void)
{
    const int N = WEI_N, M = 2 * N;
    wei_L = sqrt(N / sqrt(2.0));
    /* samples at theta_k = k pi / M, k = -M .. M-1; the k = -M sample (t = -inf) is 0 */
    for (int n = 1; n <= N; ++n) {
        double acc = 0.0;
        for (int k = -M + 1; k <= M - 1; ++k) {
            double th = k * M_PI / M;
            double t = wei_L * tan(0.5 * th);
            double f = exp(-t * t) * (wei_L * wei_L + t * t);
            acc += f * cos(n * th);
        }
        wei_a[n] = acc / (2.0 * M);
    }
    wei_ready = 1;
}

/* Re w(x + i a), a > 0. */
double ora_voigt_H(double a, double x)
{
    if (!wei_ready) wei_init();
    double complex z = x + I * a;
    double complex d = wei_L - I * z;
    double complex Z = (wei_L + I * z) / d;
    double complex p = 0.0;
    for (int n = WEI_N; n >= 1; --n) p = p * Z + wei_a[n];
    double complex w = 2.0 * p / (d * d) + (1.0 / sqrt(M_PI)) / d;
    return creal(w);
}

/* Vectorised H for the Python side. */
void ora_voigt_H_vec(int64_t n, const double* a, const double* x, double* out)
{
    if (!wei_ready) wei_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = ora_voigt_H(a[i], x[i]);
}

/* Opacity fields of one non-LTE formal solve. For wavelength index l:
 *   chi(l, c, w) = chi_c[l][c] + (line[l] >= 0 ? kappa[t][c] H(a[t][c], x) : 0)
 *   eta(l, c, w) = eta_c[l][c] + (line[l] >= 0 ? eps[t][c]   H(a[t][c], x) : 0)
 * with t = line[l] and x = (u[l] + vscale w . v[c]) / v_th[c]: u[l] = c (nu_l - nu_0)/nu_0
 * is the wavelength's velocity offset from the line centre, and the profile
 * of a ray looking along w (photons travelling along -w) is shifted by the
 * projected plasma velocity. A ray inclined at theta to the invariant axis
 * (Sec. 3.1) has the in-plane direction w of its projection and sees
 * sin(theta) of the in-plane velocity: vscale = sin(theta). */
typedef struct {
    int32_t nx, nz, n_wave, n_lines;
    const int32_t* line;   /* [n_wave] line index or -1 */
    const double* u;       /* [n_wave] m/s */
    const double* chi_c;   /* [n_wave][ncell] 1/m */
    const double* eta_c;   /* [n_wave][ncell] */
    const double* kappa;   /* [n_lines][ncell] 1/m */
    const double* eps;     /* [n_lines][ncell] */
    const double* adamp;   /* [n_lines][ncell] */
    const double* inv_vth; /* [ncell] s/m */
    const double* vx;      /* [ncell] m/s */
    const double* vz;      /* [ncell] m/s */
    double vscale;         /* velocity projection of the rays: 1 in the plane, sin(theta)
                              for rays inclined at theta to the invariant y axis */
} ora_nlte_fields;

static void nlte_opac(const void* ctx, int32_t lam, int32_t x, int32_t z, double wx, double wz,
                      double* chi, double* eta)
{
    const ora_nlte_fields* f = (const ora_nlte_fields*)ctx;
    size_t ncell = (size_t)f->nx * f->nz;
    size_t c = (size_t)z * f->nx + x;
    double ch = f->chi_c[(size_t)lam * ncell + c];
    double et = f->eta_c[(size_t)lam * ncell + c];
    int32_t t = f->line[lam];
    if (t >= 0) {
        double xx = (f->u[lam] + f->vscale * (wx * f->vx[c] + wz * f->vz[c])) * f->inv_vth[c];
        double H = ora_voigt_H(f->adamp[(size_t)t * ncell + c], xx);
        ch += f->kappa[(size_t)t * ncell + c] * H;
        et += f->eps[(size_t)t * ncell + c] * H;
    }
    *chi = ch;
    *eta = et;
}

/* Formal solve with direction-dependent line opacity. Outputs J and the
 * merged cascade-0 radiance per direction, I0[n_wave][nz][nx][N_0].
 * need_c0 (nullable): [nz][nx] mask of the cells whose J is wanted; only
 * their dependency cone is solved (J and I0 elsewhere are left 0). */
int32_t ora_nlte_formal_solve(const ora_geom* g, const ora_nlte_fields* f, const uint8_t* need_c0, double* J,
                              double* I0, int64_t* stats, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    if (!wei_ready) wei_init();
    return ora_rc_solve(g, f->n_wave, nlte_opac, f, need_c0, J, I0, stats);
}

/* Emergent intensity through the non-LTE fields (Sec. 3.9): the beam of
 * ora_emergent (light direction (wx, wz), normalised here, ray j at offset
 * j + 1/2 - n_rays/2 cells along (-wz, wx) from the domain centre), each ray
 * traced from outside the domain back along -w with the line profiles
 * shifted for that march direction. I_out[n_wave][n_rays]. */
int32_t ora_nlte_emergent(const ora_geom* g, const ora_nlte_fields* f, double wx, double wz, int32_t n_rays,
                          double* I_out)
{
    if (!wei_ready) wei_init();
    double wn = hypot(wx, wz);
    if (!(wn > 0.0)) return -1;
    wx /= wn;
    wz /= wn;
    double R = 0.5 * hypot((double)g->nx, (double)g->nz) + 2.0;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < (int64_t)f->n_wave * n_rays; ++q) {
        int32_t lam = (int32_t)(q / n_rays), j = (int32_t)(q % n_rays);
        double s = j + 0.5 - 0.5 * n_rays;
        double ox = 0.5 * g->nx + s * (-wz) + R * wx, oz = 0.5 * g->nz + s * wx + R * wz;
        double In, tau;
        ora_ray(g, nlte_opac, f, lam, ox, oz, -wx, -wz, 0.0, INFINITY, &In, &tau);
        I_out[q] = In;
    }
    return 0;
}

/* Directional opacity at the cell itself (for the cascade-0 operator):
 * out_chi[l][c][k] and the line profile H at the cell, out_H[l][c][k]
 * (0 for continuum wavelengths), for the N_0 cascade-0 directions. */
void ora_nlte_local(const ora_geom* g, const ora_nlte_fields* f, double* out_chi, double* out_H)
{
    if (!wei_ready) wei_init();
    const int32_t n0 = g->c0_dirs;
    const size_t ncell = (size_t)f->nx * f->nz;
    double wxs[64], wzs[64];
    for (int32_t k = 0; k < n0 && k < 64; ++k) ora_direction(g, 0, k, &wxs[k], &wzs[k]);
#pragma omp parallel for schedule(static)
    for (int64_t lc = 0; lc < (int64_t)f->n_wave * (int64_t)ncell; ++lc) {
        int32_t lam = (int32_t)(lc / (int64_t)ncell);
        size_t c = (size_t)(lc % (int64_t)ncell);
        int32_t x = (int32_t)(c % f->nx), z = (int32_t)(c / f->nx);
        for (int32_t k = 0; k < n0; ++k) {
            double chi, eta;
            nlte_opac(f, lam, x, z, wxs[k], wzs[k], &chi, &eta);
            out_chi[(size_t)lc * n0 + k] = chi;
            double H = 0.0;
            int32_t t = f->line[lam];
            if (t >= 0) {
                double xx = (f->u[lam] + f->vscale * (wxs[k] * f->vx[c] + wzs[k] * f->vz[c])) * f->inv_vth[c];
                H = ora_voigt_H(f->adamp[(size_t)t * ncell + c], xx);
            }
            out_H[(size_t)lc * n0 + k] = H;
        }
    }
}
