// qed_kernels.h -- kernel argument blocks and launchers shared by the kernels
// (qed_kernels.hip) and the C interface (qed_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed_device.h"

namespace qed {

constexpr int kNEnergy = 8;
constexpr int kNCount = 16;

struct SpeciesDev {
    void *x, *y, *z, *ux, *uy, *uz;
    double *tau;
    void *w, *chi;
    uint64_t *uid;
    uint32_t *n_ev;
    int64_t *count;
    int64_t cap;
    int present;
};

struct FieldDev {
    int kind;
    double E[3], B[3];
    double a0, Phi;                  // plane wave: amplitude, 2 pi n_periods
    const float *grid;
    int64_t nx, ny, nz;
    double inv_dx, inv_dy, inv_dz, x0, y0, z0;
    int n_bunches;                   // bunched plane waves
    const int64_t *offsets;
    const double *a0s, *nper;
};

struct StepDev {
    double t, dt;
    const int64_t *d_step;
    uint64_t seed;
    int rad, kmax;
    double chi_switch, gmin, chi_push_min;
    int no_recoil;
};

struct ConstsDev {
    double q, es_inv, A, tau0;
};

struct WsDev {
    uint64_t *ticket;
    LookBack lb;
    unsigned long long *status;      // [0] flags, [1..4] needed counts, [5] spare
};

struct TallyDev {
    double *energy;
    int64_t n_slots;
    int64_t *count;
};

struct PushArgs {
    TablesDev tab;
    SpeciesDev lep, pp, pr;
    FieldDev f;
    StepDev st;
    ConstsDev c;
    WsDev ws;
    TallyDev tal;
    uint64_t *uid_next;
};

struct PairArgs {
    TablesDev tab;
    SpeciesDev ph, el, po;
    FieldDev f;
    StepDev st;
    ConstsDev c;
    WsDev ws;
    TallyDev tal;
    uint64_t *uid_next;
};

struct CompactArgs {
    SpeciesDev s;
    WsDev ws;
};

hipError_t launch_push_emit(const PushArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_pair_create(const PairArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_compact(const CompactArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_init_tau(const uint64_t *uid, double *tau, const int64_t *count, uint64_t seed,
                           int n_blocks, hipStream_t s);
hipError_t launch_yee_fill(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                           const double *tperp, const double *tpar, int n_blocks, hipStream_t s);
hipError_t launch_step_advance(int64_t *d_step, hipStream_t s);

}  // namespace qed
