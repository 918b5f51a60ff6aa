// qed_fields.h -- arguments of the field solver and the deposition (qed_fields.hip).
#pragma once

#include "qed_kernels.h"

namespace qed {

struct GridGeom {
    int64_t nx, ny, nz;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    double dx, dy, dz;
};

struct DepositArgs {
    SpeciesDev s;
    const void *xo, *yo, *zo;        // start positions of [first, count), or NULL: back along u/gamma
    const int64_t *d_first;          // NULL: 0
    double q_scale;                  // charge * j_scale
    double dt;
    GridGeom g;
    float *out;                      // J [3][n] or rho [n]
    unsigned long long *skipped;     // may be NULL
};

hipError_t launch_yee_advance(float *grid, const float *J, const GridGeom &g, double dt, int n_cu, hipStream_t s);
hipError_t launch_deposit_current(const DepositArgs &a, int prec, int n_cu, hipStream_t s);
hipError_t launch_deposit_charge(const DepositArgs &a, int prec, int n_cu, hipStream_t s);
hipError_t launch_save_positions(const SpeciesDev &sp, void *xo, void *yo, void *zo, int prec, int n_cu,
                                 hipStream_t s);

}  // namespace qed
