// qed_sort.h -- arguments of the cell sort (qed_sort.hip).
#pragma once

#include <algorithm>

#include "qed_kernels.h"

namespace qed {

struct SortArgs {
    SpeciesDev src, dst;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    int64_t nx, ny, nz;
    uint32_t key_out, key_dead;     // cell keys of particles outside the grid; key of decayed photons
    int bands;                       // energy bands within a cell (1, 2, 4 or 8)
    uint32_t *key0, *key1, *idx0, *idx1, *idx_final;
    uint32_t *hist, *hoff;
    unsigned long long *live;
    WsDev ws;
};

// LSD radix passes over (key, index) pairs: the first *count entries (clamped
// to cap) of key[cur], idx[cur], 8-bit digits (digit p at bit 8p), tiles of
// 2048 keys, ping-ponging between the two buffers; returns the buffer holding
// the result.  hist and hoff hold radix_hist_len(cap) entries each.
struct RadixBufs {
    uint32_t *key[2], *idx[2];
    uint32_t *hist, *hoff;
};
int launch_radix_passes8(const RadixBufs &b, int cur, const int64_t *count, int64_t cap, int passes, int n_cu,
                         WsDev ws, hipStream_t s);
int64_t radix_hist_len(int64_t cap);

// exclusive scan of the first *count (clamped to cap) entries of in
void launch_scan_u32(const uint32_t *in, uint32_t *out, const int64_t *count, int64_t cap, int n_cu, WsDev ws,
                     hipStream_t s);

// Merging of super-particles (qed_merge.hip).
struct MergeArgs {
    SpeciesDev src, dst;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    int64_t nx, ny, nz;
    int massive, octave_min, n_octaves, sub_bins, n_dir, min_group;
    uint32_t key_out, key_dead;      // cell keys of kept-as-is particles and of decayed photons
    uint64_t seed;
    uint64_t *uid_next;
    // scratch: see launch_merge
    uint32_t *key[2], *idx[2], *mkey, *g, *o;
    uint32_t *hist, *hoff;
    int64_t *cnt;                    // live, groups, outputs, first new id
    WsDev ws;
};

// mbin_passes, cell_passes: 8-bit radix passes of the momentum-bin and cell keys
hipError_t launch_merge(MergeArgs a, int prec, int mbin_passes, int cell_passes, int n_cu, hipStream_t s);

// cell sort of keys of `bits` bits (8-bit radix passes)
hipError_t launch_sort(const SortArgs &a, int prec, int bits, int n_cu, int64_t capacity, hipStream_t s);

}  // namespace qed
