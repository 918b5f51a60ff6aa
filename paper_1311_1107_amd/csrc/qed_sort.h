// qed_sort.h -- arguments of the cell sort (qed_sort.hip).
#pragma once

#include <algorithm>

#include "qed_kernels.h"

namespace qed {

struct SortArgs {
    SpeciesDev src, dst;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    int64_t nx, ny, nz;
    uint32_t key_out, key_dead;     // keys of particles outside the grid and of decayed photons
    uint32_t *key0, *key1, *idx0, *idx1, *idx_final;
    uint32_t *hist, *hoff;
    unsigned long long *live;
    WsDev ws;
};

hipError_t launch_sort(const SortArgs &a, int prec, int passes, int n_cu, int64_t capacity, hipStream_t s);

}  // namespace qed
