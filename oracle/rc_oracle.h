/* rc_oracle.h -- declarations shared by the oracle's C files (test
 * infrastructure only; never included by the HIP library). */
#ifndef RC_ORACLE_H
#define RC_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t nx, nz;
    int32_t n_casc;
    int32_t c0_dirs;
    double t1;
    int32_t t_rule;
    int32_t bilinear_fix; /* 1: trace each merged interval to its 4 bilinear probes */
    double voxel;
} ora_geom;

typedef void (*ora_opac_fn)(const void* ctx, int32_t lam, int32_t cx, int32_t cz,
                            double wx, double wz, double* chi, double* eta);

int32_t ora_rc_solve(const ora_geom* g, int32_t n_wave, ora_opac_fn opac, const void* ctx,
                     const uint8_t* need_c0, double* J, double* I0, int64_t* stats);
void ora_direction(const ora_geom* g, int32_t i, int32_t k, double* wx, double* wz);
int32_t ora_ray(const ora_geom* g, ora_opac_fn opac, const void* ctx, int32_t lam, double cx, double cz, double wx,
                double wz, double ta, double tb, double* I_out, double* tau_out);
#endif
