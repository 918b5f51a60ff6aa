// qed_sort.hip -- stable reordering of particles by Yee-grid cell.
//
// A PIC code keeps its particles ordered by cell so that the field gather of
// neighbouring threads touches the same grid lines.  The order here is a
// stable sort by cell key, so that it is a deterministic function of the
// particle state (the oracle applies the same one): key = (i ny + j) nz + k
// of the cell holding the particle, nx ny nz for particles outside the grid,
// and the largest key for decayed photons (tau = +inf), which are dropped.
//
// LSD radix sort, 8-bit digits: per pass a count kernel (per-tile digit
// histograms, digit-major), an exclusive scan of the histograms, and a scatter
// kernel that ranks each tile in LDS in stable order and writes it out
// coalesced.  A final kernel gathers the particles into the destination
// arrays.
#include "qed_sort.h"

namespace qed {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 keys per tile

// particle count of the source, clamped to its capacity (every pass agrees on it)
__device__ __forceinline__ int64_t sort_count(const int64_t *count, int64_t cap) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

template <typename R>
__global__ void __launch_bounds__(256)
k_sort_keys(SortArgs a) {
    const int64_t n = sort_count(a.src.count, a.src.cap);
    const R *X = (const R *)a.src.x, *Y = (const R *)a.src.y, *Z = (const R *)a.src.z;
    unsigned long long live = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t key;
        if (a.src.tau[i] == HUGE_VAL) {
            key = a.key_dead;
        } else {
            ++live;
            const double gx = ((double)X[i] - a.x0) * a.inv_dx;
            const double gy = ((double)Y[i] - a.y0) * a.inv_dy;
            const double gz = ((double)Z[i] - a.z0) * a.inv_dz;
            key = a.key_out;
            if (gx >= 0.0 && gy >= 0.0 && gz >= 0.0) {
                const double fi = floor(gx), fj = floor(gy), fk = floor(gz);
                if (fi < (double)a.nx && fj < (double)a.ny && fk < (double)a.nz)
                    key = (uint32_t)(((int64_t)fi * a.ny + (int64_t)fj) * a.nz + (int64_t)fk);
            }
            if (a.bands > 1) {
                // band of |u|: floor(log2 |u|^2 / 6) in [0, bands), from the exponent of |u|^2
                const double ux = (double)((const R *)a.src.ux)[i], uy = (double)((const R *)a.src.uy)[i],
                             uz = (double)((const R *)a.src.uz)[i];
                const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
                int e = 0;
                if (u2 > 0.0 && isfinite(u2)) (void)frexp(u2, &e);
                int b = (e - 1) >= 0 ? (e - 1) / 6 : 0;
                b = b < a.bands - 1 ? b : a.bands - 1;
                key = key * (uint32_t)a.bands + (uint32_t)b;
            }
        }
        a.key0[i] = key;
        a.idx0[i] = (uint32_t)i;
    }
    live = (unsigned long long)wave_sum_u32((uint32_t)live);
    if (lane_id() == 0 && live) atomicAdd((unsigned long long *)a.live, live);
}

__global__ void k_sort_zero(unsigned long long *live) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *live = 0ull;
}

// exclusive scan of a u32 array of ceil(*count / div) * mult items
// (decoupled look-back over blocks of 4096)
__global__ void __launch_bounds__(256)
k_scan_u32(const uint32_t *in, uint32_t *out, const int64_t *count, int64_t cap, int64_t div, int64_t mult,
           WsDev ws) {
    __shared__ uint64_t s_ticket;
    __shared__ uint32_t s_wave[2 * kMaxWaves];
    __shared__ uint32_t s_pref;
    const int tid = threadIdx.x;
    const int64_t n_items = (sort_count(count, cap) + div - 1) / div * mult;
    const int64_t n_st = (n_items + kSortTile - 1) / kSortTile;
    for (;;) {
        if (tid == 0) s_ticket = atomicAdd((unsigned long long *)ws.ticket, 1ull);
        __syncthreads();
        const uint64_t tk = s_ticket;
        const uint32_t epoch = (uint32_t)(tk >> 32);
        const int64_t st = (int64_t)(tk & 0xffffffffull);
        if (st >= n_st) {
            if (tid == 0 && st == n_st + (int64_t)gridDim.x - 1)
                atomicAdd((unsigned long long *)ws.ticket,
                          (1ull << 32) - (unsigned long long)(n_st + (int64_t)gridDim.x));
            break;
        }
        const int64_t b = st * kSortTile + (int64_t)tid * kSortItems;
        uint32_t v[kSortItems], sum = 0;
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            v[j] = b + j < n_items ? in[b + j] : 0u;
            sum += v[j];
        }
        uint32_t e, e1, tot, tot1;
        block_scan2(sum, 0u, e, e1, tot, tot1, s_wave);
        if (tid < kWave) {
            uint32_t p0, p1;
            lookback2(ws.lb, st, epoch, tot, 0u, p0, p1);
            if (tid == 0) s_pref = p0;
        }
        __syncthreads();
        uint32_t r = s_pref + e;
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (b + j < n_items) out[b + j] = r;
            r += v[j];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// 8-bit digits: half the passes of the 4-bit form (three for keys of up to
// 24 bits).  Tiles of 2048 keys, eight rounds of 256.  Within a round each
// wave finds the lanes that share a lane's digit with nine ballots (the
// digit's bits and a bit for keys past the end), so a lane's rank among its
// wave's equal digits is a popcount and each distinct digit takes one LDS
// update per wave, however the digits repeat (cell-ordered keys repeat a
// lot).  Ranks are taken in key order (round, wave, lane), so the pass is
// stable.
// ------------------------------------------------------------------------
constexpr int kTile8 = 2048;
constexpr int kRounds8 = kTile8 / kSortThreads;      // 8
constexpr int kDigits8 = 256;

// lanes of the wave whose 9-bit digit d equals this lane's (every lane active)
__device__ __forceinline__ uint64_t match_digit9(uint32_t d) {
    uint64_t m = ~0ull;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

// per-tile histograms of one 8-bit digit, digit-major: hist[d * n_tiles + tile]
__global__ void __launch_bounds__(256)
k_radix_count8(const uint32_t *keys, const int64_t *count, int64_t cap, int shift, uint32_t *hist) {
    __shared__ uint32_t s_h[kDigits8];
    const int tid = threadIdx.x, lane = lane_id();
    const int64_t n = sort_count(count, cap);
    const int64_t n_tiles = (n + kTile8 - 1) / kTile8;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        s_h[tid] = 0u;                                    // one digit per thread
        __syncthreads();
        const int64_t b = tile * kTile8;
#pragma unroll
        for (int j = 0; j < kRounds8; ++j) {
            const int64_t i = b + j * kSortThreads + tid;
            const uint32_t d = i < n ? (keys[i] >> shift) & (kDigits8 - 1) : (uint32_t)kDigits8;
            const uint64_t m = match_digit9(d);
            if (d < (uint32_t)kDigits8 && lane == __ffsll((long long)m) - 1) atomicAdd(&s_h[d], (uint32_t)__popcll(m));
        }
        __syncthreads();
        hist[(int64_t)tid * n_tiles + tile] = s_h[tid];
        __syncthreads();
    }
}

// stable scatter of one 8-bit digit through LDS (coalesced loads and stores)
__global__ void __launch_bounds__(256)
k_radix_scatter8(const uint32_t *kin, const uint32_t *iin, uint32_t *kout, uint32_t *iout, const int64_t *count,
                 int64_t cap, int shift, const uint32_t *hoff) {
    __shared__ __align__(16) uint8_t s_cnt[kRounds8 * kMaxWaves * kDigits8];   // per (round, wave, digit) counts
    __shared__ uint16_t s_off[kRounds8 * kMaxWaves * kDigits8];    // their offsets within the digit's run
    __shared__ uint32_t s_k[kTile8], s_v[kTile8];
    __shared__ uint32_t s_start[kDigits8], s_go[kDigits8];
    __shared__ uint32_t s_wave[2 * kMaxWaves];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t n = sort_count(count, cap);
    const int64_t n_tiles = (n + kTile8 - 1) / kTile8;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * kTile8;
        const int nv = (int)(n - base < (int64_t)kTile8 ? n - base : (int64_t)kTile8);
        // zero the counts: 8 KB, 32 bytes per thread
        {
            uint4 *c4 = (uint4 *)s_cnt;
            c4[2 * tid] = make_uint4(0u, 0u, 0u, 0u);
            c4[2 * tid + 1] = make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t k[kRounds8], v[kRounds8], rk[kRounds8];
#pragma unroll
        for (int j = 0; j < kRounds8; ++j) {
            const int p = j * kSortThreads + tid;
            k[j] = p < nv ? kin[base + p] : 0u;
            v[j] = p < nv ? iin[base + p] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRounds8; ++j) {
            const int p = j * kSortThreads + tid;
            const uint32_t d = p < nv ? (k[j] >> shift) & (kDigits8 - 1) : (uint32_t)kDigits8;
            const uint64_t m = match_digit9(d);
            rk[j] = (uint32_t)__popcll(m & below);
            if (d < (uint32_t)kDigits8 && rk[j] == 0u) s_cnt[(j * kMaxWaves + wid) * kDigits8 + d] = (uint8_t)__popcll(m);
        }
        __syncthreads();
        // thread d: offsets of its digit's (round, wave) groups in key order, and the digit's count
        uint32_t run = 0;
#pragma unroll
        for (int g = 0; g < kRounds8 * kMaxWaves; ++g) {
            s_off[g * kDigits8 + tid] = (uint16_t)run;
            run += s_cnt[g * kDigits8 + tid];
        }
        uint32_t e, e1, tot, tot1;
        block_scan2(run, 0u, e, e1, tot, tot1, s_wave);
        s_start[tid] = e;
        s_go[tid] = hoff[(int64_t)tid * n_tiles + tile] - e;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRounds8; ++j) {
            const int p = j * kSortThreads + tid;
            if (p < nv) {
                const uint32_t d = (k[j] >> shift) & (kDigits8 - 1);
                const uint32_t pos = s_start[d] + s_off[(j * kMaxWaves + wid) * kDigits8 + d] + rk[j];
                s_k[pos] = k[j];
                s_v[pos] = v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRounds8; ++j) {
            const int p = j * kSortThreads + tid;
            if (p < nv) {
                const uint32_t key = s_k[p];
                const uint32_t g = s_go[(key >> shift) & (kDigits8 - 1)] + (uint32_t)p;
                kout[g] = key;
                iout[g] = s_v[p];
            }
        }
        __syncthreads();
    }
}

// gather the live particles into the destination, in sorted order; each
// thread keeps four gathers in flight
template <typename R>
__global__ void __launch_bounds__(256)
k_sort_permute(SortArgs a) {
    const int64_t live = (int64_t)*a.live;
    const uint32_t *idx = a.idx_final;
    const bool chi = a.src.chi != nullptr && a.dst.chi != nullptr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j0 < live; j0 += 4 * stride) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + u * stride;
            if (j >= live) break;
            const int64_t i = idx[j];
            ((R *)a.dst.x)[j] = ((const R *)a.src.x)[i];
            ((R *)a.dst.y)[j] = ((const R *)a.src.y)[i];
            ((R *)a.dst.z)[j] = ((const R *)a.src.z)[i];
            ((R *)a.dst.ux)[j] = ((const R *)a.src.ux)[i];
            ((R *)a.dst.uy)[j] = ((const R *)a.src.uy)[i];
            ((R *)a.dst.uz)[j] = ((const R *)a.src.uz)[i];
            ((R *)a.dst.w)[j] = ((const R *)a.src.w)[i];
            if (chi) ((R *)a.dst.chi)[j] = ((const R *)a.src.chi)[i];
            a.dst.tau[j] = a.src.tau[i];
            a.dst.uid[j] = a.src.uid[i];
            a.dst.n_ev[j] = a.src.n_ev[i];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.dst.count = live;
}

int launch_radix_passes8(const RadixBufs &b, int cur, const int64_t *count, int64_t cap, int passes, int n_cu,
                         WsDev ws, hipStream_t s) {
    const int64_t tiles = (cap + kTile8 - 1) / kTile8;
    const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)n_cu * 8));
    const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles * kDigits8 + kSortTile - 1) / kSortTile, n_cu));
    for (int p = 0; p < passes; ++p, cur ^= 1) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_count8, dim3(gb), dim3(256), 0, s, b.key[cur], count, cap, shift, b.hist);
        hipLaunchKernelGGL(k_scan_u32, dim3(gs), dim3(256), 0, s, b.hist, b.hoff, count, cap, (int64_t)kTile8,
                           (int64_t)kDigits8, ws);
        hipLaunchKernelGGL(k_radix_scatter8, dim3(gb), dim3(256), 0, s, b.key[cur], b.idx[cur], b.key[cur ^ 1],
                           b.idx[cur ^ 1], count, cap, shift, b.hoff);
    }
    return cur;
}

int64_t radix_hist_len(int64_t cap) { return (int64_t)kDigits8 * ((cap + kTile8 - 1) / kTile8 + 1); }

void launch_scan_u32(const uint32_t *in, uint32_t *out, const int64_t *count, int64_t cap, int n_cu, WsDev ws,
                     hipStream_t s) {
    const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + kSortTile - 1) / kSortTile, (int64_t)n_cu));
    hipLaunchKernelGGL(k_scan_u32, dim3(gs), dim3(256), 0, s, in, out, count, cap, (int64_t)1, (int64_t)1, ws);
}

hipError_t launch_sort(const SortArgs &a, int prec, int bits, int n_cu, int64_t capacity, hipStream_t s) {
    const unsigned ge = (unsigned)std::max<int64_t>(1, std::min<int64_t>((capacity + 255) / 256, (int64_t)n_cu * 16));
    hipLaunchKernelGGL(k_sort_zero, dim3(1), dim3(64), 0, s, a.live);
    if (prec == 0) hipLaunchKernelGGL((k_sort_keys<double>), dim3(ge), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_sort_keys<float>), dim3(ge), dim3(256), 0, s, a);
    RadixBufs b = {{a.key0, a.key1}, {a.idx0, a.idx1}, a.hist, a.hoff};
    const int fin = launch_radix_passes8(b, 0, a.src.count, a.src.cap, (bits + 7) / 8, n_cu, a.ws, s);
    SortArgs c = a;
    c.idx_final = b.idx[fin];
    if (prec == 0) hipLaunchKernelGGL((k_sort_permute<double>), dim3(ge), dim3(256), 0, s, c);
    else hipLaunchKernelGGL((k_sort_permute<float>), dim3(ge), dim3(256), 0, s, c);
    return hipGetLastError();
}

}  // namespace qed
