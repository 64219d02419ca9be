/*
 * rc_oracle.c -- plain FP64 CPU oracle for the radiance-cascades (RC) formal
 * solution of Osborne & Sannikov, "Radiance Cascades: A Novel
 * High-Resolution Formal Solution for Multidimensional Non-LTE Radiative
 * Transfer" (arXiv:2408.14425).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference the GPU path is
 * checked against. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never calls it. It shares no code,
 * headers, tables or constants with the HIP library.
 *
 * Every step follows the paper's description, in the paper's order:
 *   - radiance interval R_{a,b}(p, w) = [I_{b->a}, tau_{b->a}]   (Sec. 2.2, Eq. Rab)
 *   - merge operator M: near interval attenuates the far one      (Sec. 2.2.1)
 *   - cascade i covers the shell [t_i, t_{i+1}); spacing x2, directions
 *     x4, interval start x4 per level (alpha = 2)                 (Sec. 2.3, Eq. RcScalingLaw)
 *   - t_0 = 0, the top cascade runs to the domain edge            (Sec. 2.3)
 *   - cascade-0 probes at cell centres, uniform probe grid        (Sec. 3.2, Sec. 2.3)
 *   - bilinear interpolation of cascade i+1 onto probes of i,
 *     clamped at the grid edge                                    (Sec. 2.3.1, Sec. 2.5)
 *   - each ray of cascade i merges with its 2*alpha = 4 children  (Sec. 2.3.1)
 *   - iterative top-down merge                                    (Sec. 2.3.1)
 *   - optional bilinear fix: each merged interval traced once per
 *     bilinear probe, to the start of that probe's child cone      (Sec. 2.5)
 *   - piecewise-constant integration per cell, back to front      (Sec. 3.2, RTE solution)
 *   - free-space boundary: nothing enters the domain              (Sec. 3.4)
 *   - J = angular average of the merged cascade-0 radiance        (Sec. 1, Eq. J; flatland)
 *
 * Readings where the paper is ambiguous (each is listed in the design notes):
 *   - The printed merge formula has near and far swapped; the interval
 *     nearer the probe must attenuate the farther one: I = I_near +
 *     exp(-tau_near) I_far, tau = tau_near + tau_far.
 *   - Directions are cone centres theta_{i,k} = 2 pi (k + 1/2) / N_i, so the
 *     four children 4k..4k+3 of cascade i+1 nest inside cone k of cascade i.
 *   - Probe (u, v) of cascade i sits at ((u+1/2) 2^i, (v+1/2) 2^i) in cell
 *     units; there are ceil(n / 2^i) probes per axis.
 *   - t_i = t1 4^{i-1} for i >= 1 (geometric rule), or t_i = t1 (4^i-1)/3
 *     (interval lengths x4) as an option.
 *   - Children are weighted equally (1/4); edge taps are clamped, keeping the
 *     bilinear weights.
 *   - A ray is cut into segments at every crossing of the planes x = integer
 *     and z = integer; a segment belongs to the cell containing its midpoint;
 *     zero-length segments are dropped.
 *   - chi -> 0 is handled by writing the emission term as eta ds phi1(chi ds),
 *     phi1(x) = (1 - e^{-x}) / x, phi1(0) = 1.
 *   - Flatland angular quadrature: J = (1/N_0) sum_k I_0(k).
 *   - Bilinear fix: the child cone of direction k on a probe q of cascade
 *     i+1 is the cone of k's four children, so its start is q + t_{i+1} w_k;
 *     the top cascade has no cascade above and keeps its own rays; a probe
 *     below a top cascade that lies wholly outside the domain still traces
 *     its four intervals (merged with nothing).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "rc_oracle.h"

/* ora_geom fields: grid size in cells (nx, nz); number of cascades I
 * (n_casc); directions on cascade 0 (c0_dirs); start of cascade 1 in cells
 * (t1); interval rule (t_rule: 0 geometric t_i = t1 4^{i-1}, 1 lengths x4
 * t_i = t1 (4^i - 1)/3); physical length of one cell (voxel). */

/* ---------------------------------------------------------------- geometry */

/* Start of cascade i's interval, in cells (Eq. RcScalingLaw with alpha = 2). */
double ora_t_start(const ora_geom* g, int32_t i)
{
    if (i <= 0) return 0.0;
    if (i >= g->n_casc) return INFINITY;
    if (g->t_rule == 1) return g->t1 * (pow(4.0, i) - 1.0) / 3.0;
    return g->t1 * pow(4.0, i - 1);
}

int32_t ora_level_dirs(const ora_geom* g, int32_t i) { return g->c0_dirs << (2 * i); }
double ora_level_spacing(int32_t i) { return ldexp(1.0, i); }
int32_t ora_level_px(const ora_geom* g, int32_t i) { return (g->nx + (1 << i) - 1) >> i; }
int32_t ora_level_pz(const ora_geom* g, int32_t i) { return (g->nz + (1 << i) - 1) >> i; }

/* Direction k of cascade i: the centre of cone k. */
void ora_direction(const ora_geom* g, int32_t i, int32_t k, double* wx, double* wz)
{
    double th = 2.0 * M_PI * (k + 0.5) / (double)ora_level_dirs(g, i);
    *wx = cos(th);
    *wz = sin(th);
}

/* --------------------------------------------------------- segmentation */

/* Clip the ray P(t) = c + t w, t in [ta, tb), to the box [0,nx] x [0,nz]
 * (slab method), then cut it at every crossing of an integer x- or z-plane.
 * Writes segments ordered near -> far: cell indices and lengths dt (cells).
 * Returns the number of segments (0 for a ray that misses the box). */
int32_t ora_segments(double cx, double cz, double wx, double wz, double ta, double tb,
                     int32_t nx, int32_t nz, int32_t* seg_x, int32_t* seg_z, double* seg_dt,
                     int32_t max_seg)
{
    double lo = ta, hi = tb;
    /* x slab */
    if (wx != 0.0) {
        double a = (0.0 - cx) / wx, b = ((double)nx - cx) / wx;
        if (a > b) { double t = a; a = b; b = t; }
        if (a > lo) lo = a;
        if (b < hi) hi = b;
    } else if (cx < 0.0 || cx > (double)nx) {
        return 0;
    }
    /* z slab */
    if (wz != 0.0) {
        double a = (0.0 - cz) / wz, b = ((double)nz - cz) / wz;
        if (a > b) { double t = a; a = b; b = t; }
        if (a > lo) lo = a;
        if (b < hi) hi = b;
    } else if (cz < 0.0 || cz > (double)nz) {
        return 0;
    }
    if (!(lo < hi)) return 0;

    /* Crossing parameters of x = X planes, in increasing t, strictly in (lo, hi). */
    double xa = cx + lo * wx, xb = cx + hi * wx;
    int64_t x_first, x_last, x_step;
    if (wx > 0.0) { x_first = (int64_t)floor(xa) + 1; x_last = (int64_t)ceil(xb) - 1; x_step = 1; }
    else if (wx < 0.0) { x_first = (int64_t)ceil(xa) - 1; x_last = (int64_t)floor(xb) + 1; x_step = -1; }
    else { x_first = 1; x_last = 0; x_step = 1; }
    double za = cz + lo * wz, zb = cz + hi * wz;
    int64_t z_first, z_last, z_step;
    if (wz > 0.0) { z_first = (int64_t)floor(za) + 1; z_last = (int64_t)ceil(zb) - 1; z_step = 1; }
    else if (wz < 0.0) { z_first = (int64_t)ceil(za) - 1; z_last = (int64_t)floor(zb) + 1; z_step = -1; }
    else { z_first = 1; z_last = 0; z_step = 1; }

    int64_t X = x_first, Z = z_first;
    int x_more = (wx != 0.0) && ((x_step > 0) ? (X <= x_last) : (X >= x_last));
    int z_more = (wz != 0.0) && ((z_step > 0) ? (Z <= z_last) : (Z >= z_last));

    int32_t n = 0;
    double t_prev = lo;
    for (;;) {
        double tx = x_more ? ((double)X - cx) / wx : INFINITY;
        double tz = z_more ? ((double)Z - cz) / wz : INFINITY;
        double t_next;
        if (tx <= tz) {
            t_next = tx;
            X += x_step;
            x_more = (x_step > 0) ? (X <= x_last) : (X >= x_last);
        } else {
            t_next = tz;
            Z += z_step;
            z_more = (z_step > 0) ? (Z <= z_last) : (Z >= z_last);
        }
        if (!(t_next < hi)) t_next = hi;       /* last segment ends at the clip */
        if (t_next > t_prev) {                  /* drop zero-length segments */
            double tm = 0.5 * (t_prev + t_next);
            int64_t ix = (int64_t)floor(cx + tm * wx);
            int64_t iz = (int64_t)floor(cz + tm * wz);
            if (ix < 0) ix = 0;
            if (ix > nx - 1) ix = nx - 1;
            if (iz < 0) iz = 0;
            if (iz > nz - 1) iz = nz - 1;
            if (n >= max_seg) return -1;
            seg_x[n] = (int32_t)ix;
            seg_z[n] = (int32_t)iz;
            seg_dt[n] = t_next - t_prev;
            ++n;
            t_prev = t_next;
        }
        if (t_next >= hi) break;
    }
    return n;
}

/* ----------------------------------------------------- radiative transfer */

/* phi1(x) = (1 - e^{-x}) / x, with phi1(0) = 1. */
static double phi1(double x) { return x > 0.0 ? -expm1(-x) / x : 1.0; }

/* Back-to-front piecewise-constant solution along n segments ordered near ->
 * far (Sec. 3.2): starting from nothing beyond the far end, each segment
 * attenuates what lies behind it and adds its own emission. */
void ora_march(int32_t n, const double* chi, const double* eta, const double* ds,
               double* I_out, double* tau_out)
{
    double I = 0.0, tau = 0.0;
    for (int32_t s = n - 1; s >= 0; --s) {
        double dtau = chi[s] * ds[s];
        I = I * exp(-dtau) + eta[s] * ds[s] * phi1(dtau);
        tau += dtau;
    }
    *I_out = I;
    *tau_out = tau;
}

/* Merge operator M (Sec. 2.2.1): [a,b] is the near interval, [b,c] the far one. */
void ora_merge(double I_near, double tau_near, double I_far, double tau_far,
               double* I_out, double* tau_out)
{
    *I_out = I_near + exp(-tau_near) * I_far;
    *tau_out = tau_near + tau_far;
}

/* ora_opac_fn: opacity/emissivity a ray sees in a cell for wavelength index
 * lam when looking along (wx, wz) (declared in rc_oracle.h). */

typedef struct {
    const double* chi;  /* [n_wave][nz][nx] per unit length */
    const double* eta;
    int32_t nx, nz;
} ora_given_fields;

static void given_opac(const void* ctx, int32_t lam, int32_t x, int32_t z, double wx, double wz,
                       double* chi, double* eta)
{
    (void)wx;
    (void)wz;
    const ora_given_fields* f = (const ora_given_fields*)ctx;
    size_t idx = ((size_t)lam * f->nz + z) * f->nx + x;
    *chi = f->chi[idx];
    *eta = f->eta[idx];
}

/* March one ray: segments of [ta, tb) from (cx, cz) along (wx, wz), then
 * the back-to-front solution. Scratch buffers hold max_seg entries.
 * Returns the number of segments (cell steps). */
static int32_t march_ray(const ora_geom* g, ora_opac_fn opac, const void* ctx, int32_t lam,
                         double cx, double cz, double wx, double wz, double ta, double tb,
                         int32_t* sx, int32_t* sz, double* sdt, double* schi, double* seta,
                         double* sds, int32_t max_seg, double* I, double* tau)
{
    int32_t n = ora_segments(cx, cz, wx, wz, ta, tb, g->nx, g->nz, sx, sz, sdt, max_seg);
    if (n < 0) n = 0; /* cannot happen with max_seg = nx + nz + 4 */
    for (int32_t s = 0; s < n; ++s) {
        opac(ctx, lam, sx[s], sz[s], wx, wz, &schi[s], &seta[s]);
        sds[s] = sdt[s] * g->voxel;
    }
    ora_march(n, schi, seta, sds, I, tau);
    return n;
}

/* One ray with any opacity provider (scratch allocated here): the segments
 * of [ta, tb) from (cx, cz) along (wx, wz), solved back to front. Returns the
 * number of segments. */
int32_t ora_ray(const ora_geom* g, ora_opac_fn opac, const void* ctx, int32_t lam, double cx, double cz, double wx,
                double wz, double ta, double tb, double* I, double* tau)
{
    int32_t max_seg = g->nx + g->nz + 8;
    int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
    int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
    double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
    int32_t n = march_ray(g, opac, ctx, lam, cx, cz, wx, wz, ta, tb, sx, sz, buf, buf + max_seg, buf + 2 * max_seg,
                          buf + 3 * max_seg, max_seg, I, tau);
    free(sx);
    free(sz);
    free(buf);
    return n;
}

/* ------------------------------------------------------------------ merge */

/* Bilinear taps of probe coordinate c (cells) on the probe grid of cascade
 * i+1 (spacing s_up, P_up probes): q = c / s_up - 1/2, taps floor(q) and
 * floor(q)+1, each clamped into [0, P_up - 1], weights (1-f, f). */
static void bilinear_taps(double c, double s_up, int32_t P_up, int32_t tap[2], double w[2])
{
    double q = c / s_up - 0.5;
    double b = floor(q);
    double f = q - b;
    int64_t t0 = (int64_t)b, t1 = t0 + 1;
    if (t0 < 0) t0 = 0;
    if (t0 > P_up - 1) t0 = P_up - 1;
    if (t1 < 0) t1 = 0;
    if (t1 > P_up - 1) t1 = P_up - 1;
    tap[0] = (int32_t)t0;
    tap[1] = (int32_t)t1;
    w[0] = 1.0 - f;
    w[1] = f;
}

/* Merge cascade i with the already-merged cascade i+1 (Sec. 2.3.1):
 *   Itilde_i(p,k) = M( R_i(p,k), sum_taps w_x w_z (1/4) sum_j Itilde_{i+1}(tap, 4k+j) ).
 * Arrays are [n_wave][pz][px][dirs]. need (nullable) is a [pz][px] mask of
 * the probes to produce; others are left untouched. Iup == NULL means the
 * upper cascade contributes nothing. */
void ora_merge_level(const ora_geom* g, int32_t i, int32_t n_wave, const double* I_i,
                     const double* tau_i, const double* Iup, double* Iout, const uint8_t* need)
{
    int32_t px = ora_level_px(g, i), pz = ora_level_pz(g, i), nd = ora_level_dirs(g, i);
    int32_t qx = ora_level_px(g, i + 1), qz = ora_level_pz(g, i + 1), nd_up = nd * 4;
    double s = ora_level_spacing(i), s_up = ora_level_spacing(i + 1);
#pragma omp parallel for schedule(static)
    for (int64_t pidx = 0; pidx < (int64_t)n_wave * pz * px; ++pidx) {
        int32_t lam = (int32_t)(pidx / ((int64_t)pz * px));
        int32_t rem = (int32_t)(pidx % ((int64_t)pz * px));
        int32_t v = rem / px, u = rem % px;
        if (need && !need[(size_t)v * px + u]) continue;
        int32_t tx[2], tz[2];
        double wxv[2], wzv[2];
        bilinear_taps((u + 0.5) * s, s_up, qx, tx, wxv);
        bilinear_taps((v + 0.5) * s, s_up, qz, tz, wzv);
        for (int32_t k = 0; k < nd; ++k) {
            size_t me = (((size_t)lam * pz + v) * px + u) * nd + k;
            double far = 0.0;
            if (Iup) {
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        double child = 0.0;
                        size_t base = (((size_t)lam * qz + tz[a]) * qx + tx[b]) * nd_up + 4 * (size_t)k;
                        for (int j = 0; j < 4; ++j) child += Iup[base + j];
                        far += wzv[a] * wxv[b] * 0.25 * child;
                    }
            }
            double I, tau;
            ora_merge(I_i[me], tau_i[me], far, 0.0, &I, &tau);
            Iout[me] = I;
        }
    }
}

/* Bilinear fix (Sec. 2.5, the ringing artefact and its remedy): an
 * interval of cascade i below the top is traced not along its own ray but,
 * once for each of the four probes q of cascade i+1 it interpolates from,
 * from its usual start p + t_i w_k to the start q + t_{i+1} w_k of the
 * child cone on q (the cone of direction k holds the children 4k..4k+3, so
 * its centre is w_k). Each of these four intervals is merged with the
 * children of its own probe, and the four results are averaged with the
 * usual bilinear weights:
 *   Itilde_i(p,k) = sum_taps w_x w_z M( R(p + t_i w_k -> q + t_{i+1} w_k),
 *                                       (1/4) sum_j Itilde_{i+1}(q, 4k+j) ).
 * Iup == NULL means the upper cascade contributes nothing. Outputs
 * [n_wave][pz][px][dirs] merged. Returns the cell steps; counts the
 * non-empty traced rays into *n_nonempty. */
static int64_t level_fix(const ora_geom* g, int32_t i, int32_t n_wave, ora_opac_fn opac, const void* ctx,
                         const uint8_t* need, const double* Iup, double* Iout, int64_t* n_nonempty)
{
    int32_t px = ora_level_px(g, i), pz = ora_level_pz(g, i), nd = ora_level_dirs(g, i);
    int32_t qx = ora_level_px(g, i + 1), qz = ora_level_pz(g, i + 1), nd_up = nd * 4;
    double s = ora_level_spacing(i), s_up = ora_level_spacing(i + 1);
    double ta = ora_t_start(g, i), tb = ora_t_start(g, i + 1);
    int32_t max_seg = g->nx + g->nz + 8;
    int64_t steps = 0, nonempty = 0;
#pragma omp parallel reduction(+ : steps, nonempty)
    {
        int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
        double *sdt = buf, *schi = buf + max_seg, *seta = buf + 2 * max_seg, *sds = buf + 3 * max_seg;
        int64_t total = (int64_t)n_wave * pz * px * nd;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int32_t k = (int32_t)(r % nd);
            int64_t pr = r / nd;
            int32_t u = (int32_t)(pr % px);
            int32_t v = (int32_t)((pr / px) % pz);
            int32_t lam = (int32_t)(pr / ((int64_t)px * pz));
            if (need && !need[(size_t)v * px + u]) continue;
            int32_t tx[2], tz[2];
            double wxv[2], wzv[2];
            bilinear_taps((u + 0.5) * s, s_up, qx, tx, wxv);
            bilinear_taps((v + 0.5) * s, s_up, qz, tz, wzv);
            double wx, wz;
            ora_direction(g, i, k, &wx, &wz);
            /* the interval's usual start */
            double ax = (u + 0.5) * s + ta * wx, az = (v + 0.5) * s + ta * wz;
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    /* start of the child cone on tap probe (tx[b], tz[a]) */
                    double ex = (tx[b] + 0.5) * s_up + tb * wx, ez = (tz[a] + 0.5) * s_up + tb * wz;
                    double len = hypot(ex - ax, ez - az);
                    double In = 0.0, tn = 0.0;
                    if (len > 0.0) {
                        int32_t n = march_ray(g, opac, ctx, lam, ax, az, (ex - ax) / len, (ez - az) / len, 0.0,
                                              len, sx, sz, sdt, schi, seta, sds, max_seg, &In, &tn);
                        steps += n;
                        nonempty += (n > 0);
                    }
                    double far = 0.0;
                    if (Iup) {
                        size_t base = (((size_t)lam * qz + tz[a]) * qx + tx[b]) * nd_up + 4 * (size_t)k;
                        for (int j = 0; j < 4; ++j) far += Iup[base + j];
                        far *= 0.25;
                    }
                    double I, tau;
                    ora_merge(In, tn, far, 0.0, &I, &tau);
                    acc += wzv[a] * wxv[b] * I;
                }
            Iout[r] = acc;
        }
        free(sx);
        free(sz);
        free(buf);
    }
    if (n_nonempty) *n_nonempty += nonempty;
    return steps;
}

/* Raw (unmerged) intervals of cascade i for the probes in need (nullable).
 * Outputs [n_wave][pz][px][dirs]. Returns the number of cell steps taken. */
static int64_t level_raw(const ora_geom* g, int32_t i, int32_t n_wave, ora_opac_fn opac,
                         const void* ctx, const uint8_t* need, double* I_out, double* tau_out,
                         int64_t* n_nonempty)
{
    int32_t px = ora_level_px(g, i), pz = ora_level_pz(g, i), nd = ora_level_dirs(g, i);
    double s = ora_level_spacing(i);
    double ta = ora_t_start(g, i), tb = ora_t_start(g, i + 1);
    int32_t max_seg = g->nx + g->nz + 8;
    int64_t steps = 0, nonempty = 0;
#pragma omp parallel reduction(+ : steps, nonempty)
    {
        int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
        double *sdt = buf, *schi = buf + max_seg, *seta = buf + 2 * max_seg, *sds = buf + 3 * max_seg;
        int64_t total = (int64_t)n_wave * pz * px * nd;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int32_t k = (int32_t)(r % nd);
            int64_t pr = r / nd;
            int32_t u = (int32_t)(pr % px);
            int32_t v = (int32_t)((pr / px) % pz);
            int32_t lam = (int32_t)(pr / ((int64_t)px * pz));
            if (need && !need[(size_t)v * px + u]) continue;
            double wx, wz;
            ora_direction(g, i, k, &wx, &wz);
            double I, tau;
            int32_t n = march_ray(g, opac, ctx, lam, (u + 0.5) * s, (v + 0.5) * s, wx, wz, ta, tb,
                                  sx, sz, sdt, schi, seta, sds, max_seg, &I, &tau);
            I_out[r] = I;
            tau_out[r] = tau;
            steps += n;
            nonempty += (n > 0);
        }
        free(sx);
        free(sz);
        free(buf);
    }
    if (n_nonempty) *n_nonempty += nonempty;
    return steps;
}

/* Full RC solve with an arbitrary opacity provider.
 *   need_c0 (nullable): [nz][nx] mask of the cascade-0 probes (cells) whose J
 *     is wanted; only their dependency cone is computed (others untouched).
 *   J: [n_wave][nz][nx];  I0 (nullable): merged cascade 0, [n_wave][nz][nx][N_0].
 *   stats (nullable): [0] rays marched, [1] non-empty rays, [2] cell steps. */
int32_t ora_rc_solve(const ora_geom* g, int32_t n_wave, ora_opac_fn opac, const void* ctx,
                     const uint8_t* need_c0, double* J, double* I0, int64_t* stats)
{
    int32_t I = g->n_casc;
    if (I < 1 || g->nx < 1 || g->nz < 1 || n_wave < 1) return -1;
    /* Dependency cone, bottom-up: the probes of i+1 that feed needed probes of i. */
    uint8_t** need = (uint8_t**)calloc((size_t)I, sizeof(uint8_t*));
    for (int32_t i = 0; i < I; ++i) {
        size_t np = (size_t)ora_level_px(g, i) * ora_level_pz(g, i);
        need[i] = (uint8_t*)calloc(np, 1);
    }
    {
        size_t np0 = (size_t)g->nx * g->nz;
        for (size_t p = 0; p < np0; ++p) need[0][p] = need_c0 ? need_c0[p] : 1;
    }
    for (int32_t i = 0; i + 1 < I; ++i) {
        int32_t px = ora_level_px(g, i), pz = ora_level_pz(g, i);
        int32_t qx = ora_level_px(g, i + 1), qz = ora_level_pz(g, i + 1);
        double s = ora_level_spacing(i), s_up = ora_level_spacing(i + 1);
        for (int32_t v = 0; v < pz; ++v)
            for (int32_t u = 0; u < px; ++u) {
                if (!need[i][(size_t)v * px + u]) continue;
                int32_t tx[2], tz[2];
                double w[2];
                bilinear_taps((u + 0.5) * s, s_up, qx, tx, w);
                bilinear_taps((v + 0.5) * s, s_up, qz, tz, w);
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) need[i + 1][(size_t)tz[a] * qx + tx[b]] = 1;
            }
    }

    int64_t rays = 0, nonempty = 0, steps = 0;
    double* up = NULL; /* merged cascade i+1 */
    for (int32_t i = I - 1; i >= 0; --i) {
        size_t n = (size_t)n_wave * ora_level_px(g, i) * ora_level_pz(g, i) * ora_level_dirs(g, i);
        double* merged = (double*)calloc(n, sizeof(double));
        const int fix = g->bilinear_fix && i < I - 1;
        {
            int64_t cnt = 0;
            size_t np = (size_t)ora_level_px(g, i) * ora_level_pz(g, i);
            for (size_t p = 0; p < np; ++p) cnt += need[i][p];
            rays += cnt * (int64_t)ora_level_dirs(g, i) * n_wave * (fix ? 4 : 1);
        }
        if (fix) {
            /* four traced intervals per merged one (Sec. 2.5) */
            steps += level_fix(g, i, n_wave, opac, ctx, need[i], up, merged, &nonempty);
            free(up);
            up = merged;
            continue;
        }
        double* raw_I = (double*)calloc(n, sizeof(double));
        double* raw_tau = (double*)calloc(n, sizeof(double));
        steps += level_raw(g, i, n_wave, opac, ctx, need[i], raw_I, raw_tau, &nonempty);
        if (i == I - 1) {
            memcpy(merged, raw_I, n * sizeof(double)); /* top cascade: nothing beyond */
        } else {
            ora_merge_level(g, i, n_wave, raw_I, raw_tau, up, merged, need[i]);
        }
        free(raw_I);
        free(raw_tau);
        free(up);
        up = merged;
    }
    /* J at cascade 0 (flatland): average over the N_0 merged directions. */
    int32_t nd0 = g->c0_dirs;
    for (int32_t lam = 0; lam < n_wave; ++lam)
        for (int32_t z = 0; z < g->nz; ++z)
            for (int32_t x = 0; x < g->nx; ++x) {
                size_t cell = (size_t)z * g->nx + x;
                if (!need[0][cell]) continue;
                size_t base = (((size_t)lam * g->nz + z) * g->nx + x) * nd0;
                double acc = 0.0;
                for (int32_t k = 0; k < nd0; ++k) acc += up[base + k];
                J[((size_t)lam * g->nz + z) * g->nx + x] = acc / nd0;
                if (I0)
                    for (int32_t k = 0; k < nd0; ++k) I0[base + k] = up[base + k];
            }
    free(up);
    for (int32_t i = 0; i < I; ++i) free(need[i]);
    free(need);
    if (stats) {
        stats[0] = rays;
        stats[1] = nonempty;
        stats[2] = steps;
    }
    return 0;
}

/* GivenFs formal solve: isotropic chi, eta [n_wave][nz][nx] -> J. */
int32_t ora_formal_solve(const ora_geom* g, int32_t n_wave, const double* chi, const double* eta,
                         const uint8_t* need_c0, double* J, double* I0, int64_t* stats,
                         int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    ora_given_fields f = {chi, eta, g->nx, g->nz};
    return ora_rc_solve(g, n_wave, given_opac, &f, need_c0, J, I0, stats);
}

/* Raw intervals of one cascade for the GivenFs fields (for checking the
 * interval geometry in isolation). Outputs [n_wave][pz][px][dirs]. */
int64_t ora_level_intervals(const ora_geom* g, int32_t i, int32_t n_wave, const double* chi,
                            const double* eta, double* I_out, double* tau_out)
{
    ora_given_fields f = {chi, eta, g->nx, g->nz};
    return level_raw(g, i, n_wave, given_opac, &f, NULL, I_out, tau_out, NULL);
}

/* Long characteristics, the brute-force reference: from every cell centre,
 * M rays at theta_m = 2 pi (m + 1/2) / M run to the domain edge; J is their
 * average. This measures the method's own error, not parity. */
int32_t ora_lc_solve(int32_t nx, int32_t nz, double voxel, int32_t M, int32_t n_wave,
                     const double* chi, const double* eta, double* J, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    ora_geom g;
    memset(&g, 0, sizeof(g));
    g.nx = nx;
    g.nz = nz;
    g.n_casc = 1;
    g.c0_dirs = M;
    g.voxel = voxel;
    ora_given_fields f = {chi, eta, nx, nz};
    int32_t max_seg = nx + nz + 8;
#pragma omp parallel
    {
        int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
        double *sdt = buf, *schi = buf + max_seg, *seta = buf + 2 * max_seg, *sds = buf + 3 * max_seg;
#pragma omp for schedule(dynamic, 16)
        for (int64_t c = 0; c < (int64_t)n_wave * nx * nz; ++c) {
            int32_t lam = (int32_t)(c / ((int64_t)nx * nz));
            int32_t rem = (int32_t)(c % ((int64_t)nx * nz));
            int32_t z = rem / nx, x = rem % nx;
            double acc = 0.0;
            for (int32_t m = 0; m < M; ++m) {
                double th = 2.0 * M_PI * (m + 0.5) / M;
                double I, tau;
                march_ray(&g, given_opac, &f, lam, x + 0.5, z + 0.5, cos(th), sin(th), 0.0, INFINITY,
                          sx, sz, sdt, schi, seta, sds, max_seg, &I, &tau);
                acc += I;
            }
            J[c] = acc / M;
        }
        free(sx);
        free(sz);
        free(buf);
    }
    return 0;
}

/* Emergent intensity along parallel long characteristics (Sec. 3.9): a beam
 * of n_rays rays of light direction (wx, wz) (normalised here), one cell
 * apart across the beam and centred on the domain, ray j at offset
 * j + 1/2 - n_rays/2 cells along (-wz, wx); each is traced from outside the
 * domain on the observer's side back along -w through the whole domain,
 * nothing entering from behind. I: [n_wave][n_rays]. */
int32_t ora_emergent(int32_t nx, int32_t nz, double voxel, int32_t n_wave, const double* chi, const double* eta,
                     double wx, double wz, int32_t n_rays, double* I, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    double wn = hypot(wx, wz);
    if (!(wn > 0.0)) return -1;
    wx /= wn;
    wz /= wn;
    ora_geom g;
    memset(&g, 0, sizeof(g));
    g.nx = nx;
    g.nz = nz;
    g.n_casc = 1;
    g.c0_dirs = 4;
    g.voxel = voxel;
    ora_given_fields f = {chi, eta, nx, nz};
    int32_t max_seg = nx + nz + 8;
    double R = 0.5 * hypot((double)nx, (double)nz) + 2.0;
#pragma omp parallel
    {
        int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
        double *sdt = buf, *schi = buf + max_seg, *seta = buf + 2 * max_seg, *sds = buf + 3 * max_seg;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < (int64_t)n_wave * n_rays; ++q) {
            int32_t lam = (int32_t)(q / n_rays), j = (int32_t)(q % n_rays);
            double s = j + 0.5 - 0.5 * n_rays;
            double ox = 0.5 * nx + s * (-wz) + R * wx, oz = 0.5 * nz + s * wx + R * wz;
            double In, tau;
            march_ray(&g, given_opac, &f, lam, ox, oz, -wx, -wz, 0.0, INFINITY, sx, sz, sdt, schi, seta, sds,
                      max_seg, &In, &tau);
            I[q] = In;
        }
        free(sx);
        free(sz);
        free(buf);
    }
    return 0;
}

/* Long characteristics at selected cells only: J at (px[q], pz[q], lam[q]). */
int32_t ora_lc_points(int32_t nx, int32_t nz, double voxel, int32_t M, int32_t n_wave,
                      const double* chi, const double* eta, int32_t n_pts, const int32_t* px,
                      const int32_t* pz, const int32_t* plam, double* J, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    (void)n_wave;
    ora_geom g;
    memset(&g, 0, sizeof(g));
    g.nx = nx;
    g.nz = nz;
    g.n_casc = 1;
    g.c0_dirs = M;
    g.voxel = voxel;
    ora_given_fields f = {chi, eta, nx, nz};
    int32_t max_seg = nx + nz + 8;
    for (int32_t q = 0; q < n_pts; ++q) {
        double acc = 0.0;
#pragma omp parallel reduction(+ : acc)
        {
            int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * max_seg);
            int32_t* sz = (int32_t*)malloc(sizeof(int32_t) * max_seg);
            double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)max_seg);
            double *sdt = buf, *schi = buf + max_seg, *seta = buf + 2 * max_seg, *sds = buf + 3 * max_seg;
#pragma omp for schedule(static)
            for (int32_t m = 0; m < M; ++m) {
                double th = 2.0 * M_PI * (m + 0.5) / M;
                double I, tau;
                march_ray(&g, given_opac, &f, plam[q], px[q] + 0.5, pz[q] + 0.5, cos(th), sin(th),
                          0.0, INFINITY, sx, sz, sdt, schi, seta, sds, max_seg, &I, &tau);
                acc += I;
            }
            free(sx);
            free(sz);
            free(buf);
        }
        J[q] = acc / M;
    }
    return 0;
}

int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
