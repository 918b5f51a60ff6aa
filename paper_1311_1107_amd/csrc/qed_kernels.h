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
    double a0, Phi, inv_Phi;         // plane wave: amplitude, 2 pi n_periods, its reciprocal
    const float *grid;
    int64_t nx, ny, nz;
    double inv_dx, inv_dy, inv_dz, x0, y0, z0;
    const float *bound;              // Yee: per-block |E|, |B| bounds (photon-step cull) or NULL
    int64_t bb, nbx, nby, nbz;       // cells per block edge, blocks per axis
    int n_bunches;                   // bunched plane waves
    const int64_t *offsets;
    const double *a0s, *nper;
    int lds_bunches;                 // the bunch table fits kLdsBunchBytes: staged in LDS
};

// Bunch table staged in LDS by the lepton step of the batched form (offsets,
// amplitudes, phase lengths and their reciprocals): 8 (n + 1) + 24 n bytes
// for n bunches.
constexpr int kLdsBunchBytes = 16384;
__host__ __device__ constexpr int64_t lds_bunch_bytes(int64_t n) { return 8 * (n + 1) + 24 * n; }

struct StepDev {
    double t, dt;
    const int64_t *d_step;
    uint64_t seed;
    int rad, kmax;
    double chi_switch, gmin, chi_push_min;
    int no_recoil;
    int variants;                    // VAR_* bits
};

enum { VAR_SOKOLOV_G = 1, VAR_PAIR_MOMENTUM = 2 };

struct ConstsDev {
    double q, es_inv, A, tau0;
};

// Event items written by the stream pass of the lepton step for its event
// pass: one record per particle whose optical depth runs out in the step, at
// slot tile * 64 + rank (tiles of one wave), so that the items of a tile are
// adjacent.  A record is whole 16-byte words (80 bytes in FP32, 144 in FP64):
// the event pass reads each with a few wide loads.
constexpr int kItemReals = 16;
template <typename R>
struct alignas(16) ItemRec {
    R v[kItemReals];     // 0-2 position x^n, 3-5 u after the push, 6-8 E, 9-11 B,
                         // 12 gamma after the push, 13 chi_e, 14 emission rate W, 15 weight
    double tau;          // optical depth at the start of the step
    uint32_t idx;        // index of the particle
    uint32_t pad;
};
static_assert(sizeof(ItemRec<float>) == 80 && sizeof(ItemRec<double>) == 144, "item record layout");
constexpr int64_t kItemBytes = sizeof(ItemRec<double>);
// Emission records written by the event pass for the append pass: one per
// event item, in item order (dense).  Reals (SoA, stride `slots`): 0-2
// position x^n, 3-5 direction u_hat, 6 weight, 7-10 gamma_gamma of each event,
// 11-14 chi_gamma of each event.
constexpr int kRecReals = 15;
struct StageDev {
    void *item;                      // ItemRec<double> or ItemRec<float> per slot
    uint32_t *item_map;              // item d (dense, in particle order) -> its slot
    void *rec;                       // kRecReals * slots reals (double or float)
    uint32_t *meta;                  // per record: events (bits 0-2), destination of event k (2 bits at 3+2k)
    uint32_t *n_rec;                 // per chunk of 64 records
    int64_t slots;
};

// Written by the scan passes for the passes after them in the same launch.
struct LaunchInfo {
    int64_t base0, base1;            // counts of the two destination buffers before the launch
    uint64_t uid0;                   // first id handed out by the launch
    int64_t n_items;                 // event items of the lepton step
};

struct WsDev {
    uint64_t *ticket;
    LookBack lb;
    unsigned long long *status;      // [0] flags, [1..4] needed counts, [5] spare
    uint32_t *tile_cnt0, *tile_cnt1; // per physics tile: appends to buffers 0 and 1
    uint32_t *tile_pre0, *tile_pre1; // their exclusive prefixes over tiles
    LaunchInfo *info;
    StageDev stage;
    int64_t max_tiles;
};

struct TallyDev {
    double *energy;
    int64_t n_slots;
    int64_t *count;
};

struct PushArgs {
    TablesDev tab;
    int64_t tile_sz;                 // tile of the physics pass (its block size)
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
    int64_t tile_sz;                 // tile of the physics pass: one wave (64 photons)
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

// Scan pass: prefixes of the per-tile append counts of the physics pass that
// ran over *src_count units with tiles of tile_sz; mode 0 appends photons
// (buffer 0 pushed, buffer 1 recorded, one id each), mode 1 appends pairs
// (one electron in buffer 0 and one positron in buffer 1 per event, two ids),
// mode 2 lists the lepton step's event items (item_map, info->n_items).
struct ScanArgs {
    const int64_t *src_count;
    int64_t tile_sz;
    SpeciesDev d0, d1;
    uint64_t *uid_next;
    int mode;
    WsDev ws;
};

hipError_t launch_lepton_stream(const PushArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_lepton_events(const PushArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_pair_create(const PairArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_scan_tiles(const ScanArgs &a, dim3 grid, hipStream_t s);
hipError_t launch_push_append(const PushArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_pair_append(const PairArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_compact(const CompactArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_init_tau(const uint64_t *uid, double *tau, const int64_t *count, uint64_t seed,
                           int n_blocks, hipStream_t s);
hipError_t launch_field_bound(const float *grid, int64_t nx, int64_t ny, int64_t nz, int64_t block, float *bound,
                              hipStream_t s);
hipError_t launch_yee_fill(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                           const double *tperp, const double *tpar, int n_blocks, hipStream_t s);
hipError_t launch_step_advance(int64_t *d_step, hipStream_t s);

struct SpectrumArgs {
    SpeciesDev s;
    int photons, n_bins;
    double ln_emin, inv_dln, e_min, e_max, wscale;
    unsigned long long *count, *wsum;
};
hipError_t launch_spectrum(const SpectrumArgs &a, int prec, int n_blocks, hipStream_t s);

}  // namespace qed
