// qed_merge.hip -- merging of super-particles (coalescence).
//
// The paper requires only that merging keep energy and momentum (end of
// Sec. 3).  Particles are grouped by (cell, energy bin, direction bin) and a
// group of at least min_group members becomes two particles that keep its
// weight, momentum and energy exactly: the two-particle merge of Vranic et al.
// (Comput. Phys. Commun. 191, 65 (2015)).
//
// Pipeline (no host synchronisation; every count stays on the device):
//   keys     cell key and momentum bin of every particle, the live count;
//   sort     stable LSD radix sort by momentum bin, then by cell key, so the
//            order is (cell, momentum bin, input index);
//   heads    group heads in sorted order, scanned into group ids;
//   starts   first sorted position of every group, and the group count;
//   sizes    output size of every group (2 if merged, else its size),
//            scanned into output offsets;
//   total    output count, the first new id, the id counter advanced;
//   copy     members of unmerged groups, one thread per particle;
//   groups   one wave per merged group: two passes of FP64 sums over its
//            members, then the two new particles.
// Key decisions are taken in FP64 with the same operations as the oracle:
// |u|^2 = fma(uz, uz, fma(uy, uy, ux ux)), frexp for the octave, correctly
// rounded division for the face coordinates, so groups are bit-identical.
#include "qed_sort.h"

namespace qed {

__global__ void k_merge_zero(int64_t *cnt) {
    if (threadIdx.x < 4 && blockIdx.x == 0) cnt[threadIdx.x] = 0;
}

__device__ __forceinline__ int64_t merge_count(const int64_t *count, int64_t cap) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

// momentum bin of u, or -1 if |u|^2 is outside the energy range; d = face axis
__device__ __forceinline__ int64_t merge_mbin(const MergeArgs &a, double ux, double uy, double uz, int &d) {
    const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
    d = 0;
    if (!(u2 > 0.0) || !isfinite(u2)) return -1;
    int ex;
    const double man = frexp(u2, &ex);
    const int64_t oct = (int64_t)ex - 1 - a.octave_min;
    if (oct < 0 || oct >= a.n_octaves) return -1;
    const int64_t sub = (int64_t)floor((2.0 * man - 1.0) * (double)a.sub_bins);
    const double ax = fabs(ux), ay = fabs(uy), az = fabs(uz);
    double ud = ax, ua = uy, ub = uz, sd = ux;
    if (ay > ud) { d = 1; ud = ay; ua = uz; ub = ux; sd = uy; }
    if (az > ud) { d = 2; ud = az; ua = ux; ub = uy; sd = uz; }
    const double h = 0.5 * (double)a.n_dir;
    int64_t ia = (int64_t)floor((ua / ud + 1.0) * h);
    int64_t ib = (int64_t)floor((ub / ud + 1.0) * h);
    ia = ia < 0 ? 0 : (ia > a.n_dir - 1 ? a.n_dir - 1 : ia);
    ib = ib < 0 ? 0 : (ib > a.n_dir - 1 ? a.n_dir - 1 : ib);
    const int64_t face = 2 * d + (sd < 0.0 ? 1 : 0);
    return ((oct * a.sub_bins + sub) * 6 + face) * ((int64_t)a.n_dir * a.n_dir) + ia * a.n_dir + ib;
}

template <typename R>
__global__ void __launch_bounds__(256)
k_merge_keys(MergeArgs a) {
    const int64_t n = merge_count(a.src.count, a.src.cap);
    const R *X = (const R *)a.src.x, *Y = (const R *)a.src.y, *Z = (const R *)a.src.z;
    const R *UX = (const R *)a.src.ux, *UY = (const R *)a.src.uy, *UZ = (const R *)a.src.uz;
    const R *Wt = (const R *)a.src.w;
    uint32_t live = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t ck = a.key_dead, mk = 0;
        if (a.src.tau[i] != HUGE_VAL) {
            ++live;
            ck = a.key_out;
            const double gx = ((double)X[i] - a.x0) * a.inv_dx;
            const double gy = ((double)Y[i] - a.y0) * a.inv_dy;
            const double gz = ((double)Z[i] - a.z0) * a.inv_dz;
            uint32_t cell = a.key_out;
            if (gx >= 0.0 && gy >= 0.0 && gz >= 0.0) {
                const double fi = floor(gx), fj = floor(gy), fk = floor(gz);
                if (fi < (double)a.nx && fj < (double)a.ny && fk < (double)a.nz)
                    cell = (uint32_t)(((int64_t)fi * a.ny + (int64_t)fj) * a.nz + (int64_t)fk);
            }
            int d;
            const int64_t mb = merge_mbin(a, (double)UX[i], (double)UY[i], (double)UZ[i], d);
            const double w = (double)Wt[i];
            if (cell != a.key_out && mb >= 0 && w > 0.0 && isfinite(w)) {
                ck = cell;
                mk = (uint32_t)mb;
            }
        }
        a.key[0][i] = mk;
        a.idx[0][i] = (uint32_t)i;
        a.g[i] = ck;
        a.mkey[i] = mk;
    }
    live = wave_sum_u32(live);
    if (lane_id() == 0 && live) atomicAdd((unsigned long long *)&a.cnt[0], (unsigned long long)live);
}

// stage-2 keys: the cell key of the particle now at each position
__global__ void __launch_bounds__(256)
k_merge_rekey(const uint32_t *ckey, const uint32_t *idx, uint32_t *key, const int64_t *count, int64_t cap) {
    const int64_t n = merge_count(count, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        key[i] = ckey[idx[i]];
}

// head[i] = 1 where a group starts; every kept-as-is particle is its own group
__global__ void __launch_bounds__(256)
k_merge_heads(const uint32_t *kf, const uint32_t *idx, const uint32_t *mkey, uint32_t key_out,
              const int64_t *cnt, uint32_t *head) {
    const int64_t live = cnt[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < live; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = kf[i];
        uint32_t h = 1u;
        if (i > 0 && k != key_out && k == kf[i - 1] && mkey[idx[i]] == mkey[idx[i - 1]]) h = 0u;
        head[i] = h;
    }
}

__global__ void __launch_bounds__(256)
k_merge_starts(const uint32_t *head, const uint32_t *hscan, int64_t *cnt, uint32_t *gstart) {
    const int64_t live = cnt[0];
    if (live == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        cnt[1] = 0;
        gstart[0] = 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < live; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = head[i], g = hscan[i];
        if (h) gstart[g] = (uint32_t)i;
        if (i == live - 1) {
            cnt[1] = (int64_t)(g + h);
            gstart[g + h] = (uint32_t)live;
        }
    }
}

__global__ void __launch_bounds__(256)
k_merge_sizes(const uint32_t *gstart, const int64_t *cnt, int min_group, uint32_t *osz) {
    const int64_t ng = cnt[1];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t sz = gstart[g + 1] - gstart[g];
        osz[g] = sz >= (uint32_t)min_group ? 2u : sz;
    }
}

__global__ void k_merge_total(const uint32_t *osz, const uint32_t *ooff, int64_t *cnt, uint64_t *uid_next,
                              int64_t *dst_count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t ng = cnt[1];
    const int64_t tot = ng > 0 ? (int64_t)ooff[ng - 1] + (int64_t)osz[ng - 1] : 0;
    const uint64_t base = *uid_next;
    cnt[2] = tot;
    cnt[3] = (int64_t)base;
    *uid_next = base + (uint64_t)tot;
    *dst_count = tot;
}

template <typename R>
__global__ void __launch_bounds__(256)
k_merge_copy(MergeArgs a, const uint32_t *idx, const uint32_t *head, const uint32_t *hscan, const uint32_t *gstart,
             const uint32_t *ooff) {
    const int64_t live = a.cnt[0];
    const bool chi = a.src.chi != nullptr && a.dst.chi != nullptr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < live; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = hscan[i] + head[i] - 1u;
        const uint32_t g0 = gstart[g];
        if (gstart[g + 1] - g0 >= (uint32_t)a.min_group) continue;
        const int64_t j = (int64_t)ooff[g] + (i - (int64_t)g0);
        const int64_t s = idx[i];
        ((R *)a.dst.x)[j] = ((const R *)a.src.x)[s];
        ((R *)a.dst.y)[j] = ((const R *)a.src.y)[s];
        ((R *)a.dst.z)[j] = ((const R *)a.src.z)[s];
        ((R *)a.dst.ux)[j] = ((const R *)a.src.ux)[s];
        ((R *)a.dst.uy)[j] = ((const R *)a.src.uy)[s];
        ((R *)a.dst.uz)[j] = ((const R *)a.src.uz)[s];
        ((R *)a.dst.w)[j] = ((const R *)a.src.w)[s];
        if (chi) ((R *)a.dst.chi)[j] = ((const R *)a.src.chi)[s];
        a.dst.tau[j] = a.src.tau[s];
        a.dst.uid[j] = a.src.uid[s];
        a.dst.n_ev[j] = a.src.n_ev[s];
    }
}

template <typename R>
__device__ __noinline__ void merge_write(const MergeArgs &a, int64_t o, uint64_t base, double sw, double un,
                                         double gap, double hx, double hy, double hz, int d, double sx, double sy,
                                         double sz, double sc, bool chi);

// one wave per merged group
template <typename R>
__global__ void __launch_bounds__(256)
k_merge_groups(MergeArgs a, const uint32_t *idx, const uint32_t *gstart, const uint32_t *ooff) {
    const int64_t ng = a.cnt[1];
    const uint64_t base = (uint64_t)a.cnt[3];
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const R *X = (const R *)a.src.x, *Y = (const R *)a.src.y, *Z = (const R *)a.src.z;
    const R *UX = (const R *)a.src.ux, *UY = (const R *)a.src.uy, *UZ = (const R *)a.src.uz;
    const R *Wt = (const R *)a.src.w, *CH = (const R *)a.src.chi;
    const bool chi = CH != nullptr && a.dst.chi != nullptr;
    const bool massive = a.massive != 0;
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; g < ng; g += waves) {
        const uint32_t b0 = gstart[g], b1 = gstart[g + 1];
        if (b1 - b0 < (uint32_t)a.min_group) continue;
        // energies relative to the first member: identical particles give back their momentum
        const int64_t i0 = idx[b0];
        const double u0x = (double)UX[i0], u0y = (double)UY[i0], u0z = (double)UZ[i0];
        const double m0 = sqrt(u0x * u0x + u0y * u0y + u0z * u0z);
        const double e0 = massive ? sqrt(1.0 + m0 * m0) : m0;
        double sw = 0.0, px = 0.0, py = 0.0, pz = 0.0, se = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, sc = 0.0;
        for (uint32_t j = b0 + lane; j < b1; j += kWave) {
            const int64_t i = idx[j];
            const double w = (double)Wt[i], ux = (double)UX[i], uy = (double)UY[i], uz = (double)UZ[i];
            const double mi = sqrt(ux * ux + uy * uy + uz * uz);
            const double ei = massive ? sqrt(1.0 + mi * mi) : mi;
            sw += w;
            px += w * ux; py += w * uy; pz += w * uz;
            se += w * (ei - e0);
            sx += w * (double)X[i]; sy += w * (double)Y[i]; sz += w * (double)Z[i];
            if (chi) sc += w * (double)CH[i];
        }
        sw = wave_sum_f64(sw);
        px = wave_sum_f64(px); py = wave_sum_f64(py); pz = wave_sum_f64(pz);
        se = wave_sum_f64(se);
        sx = wave_sum_f64(sx); sy = wave_sum_f64(sy); sz = wave_sum_f64(sz);
        sc = wave_sum_f64(sc);
        int d;
        (void)merge_mbin(a, u0x, u0y, u0z, d);
        const double sew = se / sw;
        const double eps = e0 + sew;                       // energy per unit weight
        double un = eps;                                   // |u_new|
        if (massive) {
            const double ur = sqrt(fmax((eps - 1.0) * (eps + 1.0), 0.0));
            un = (ur + m0 > 0.0) ? m0 + sew * (eps + e0) / (ur + m0) : 0.0;
        }
        const double pn = sqrt(px * px + py * py + pz * pz);
        double hx = 0.0, hy = 0.0, hz = 0.0;
        if (pn > 0.0) {
            hx = px / pn; hy = py / pn; hz = pz / pn;
        } else {
            hx = d == 0 ? 1.0 : 0.0; hy = d == 1 ? 1.0 : 0.0; hz = d == 2 ? 1.0 : 0.0;
        }
        // gap W |u_new| - |P| = sum w (|u_new| - |u|) + sum w |u| |u_hat - P_hat|^2 / 2
        double gap = 0.0;
        for (uint32_t j = b0 + lane; j < b1; j += kWave) {
            const int64_t i = idx[j];
            const double w = (double)Wt[i], ux = (double)UX[i], uy = (double)UY[i], uz = (double)UZ[i];
            const double mi = sqrt(ux * ux + uy * uy + uz * uz);
            if (massive) gap += w * (un - mi);
            if (mi > 0.0) {
                const double qx = ux / mi - hx, qy = uy / mi - hy, qz = uz / mi - hz;
                gap += w * mi * 0.5 * (qx * qx + qy * qy + qz * qz);
            }
        }
        gap = wave_sum_f64(gap);
        if (lane == 0) merge_write<R>(a, ooff[g], base, sw, un, gap, hx, hy, hz, d, sx, sy, sz, sc, chi);
    }
}

// the two new particles of a group at dst[o], dst[o + 1]
template <typename R>
__device__ __noinline__ void merge_write(const MergeArgs &a, int64_t o, uint64_t base, double sw, double un,
                                         double gap, double hx, double hy, double hz, int d, double sx, double sy,
                                         double sz, double sc, bool chi) {
    double omc = (sw * un > 0.0) ? gap / (sw * un) : 0.0;      // 1 - cos theta
    omc = omc < 0.0 ? 0.0 : (omc > 1.0 ? 1.0 : omc);
    const double ct = 1.0 - omc;
    const double st = sqrt(omc * (1.0 + ct));
    // n = P_hat x e_(d+1), normalised.  Written as the full cross product
    // with a 0/1 vector, without branches: a branchy form of this selection
    // came out of the compiler with the z-face component lost.
    const double ex = d == 2 ? 1.0 : 0.0, ey = d == 0 ? 1.0 : 0.0, ez = d == 1 ? 1.0 : 0.0;
    double nx = hy * ez - hz * ey, ny = hz * ex - hx * ez, nz = hx * ey - hy * ex;
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nn; ny /= nn; nz /= nn;
    const R xm = (R)(sx / sw), ym = (R)(sy / sw), zm = (R)(sz / sw), wh = (R)(0.5 * sw);
    for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? 1.0 : -1.0;
        const int64_t j = o + side;
        ((R *)a.dst.x)[j] = xm;
        ((R *)a.dst.y)[j] = ym;
        ((R *)a.dst.z)[j] = zm;
        ((R *)a.dst.ux)[j] = (R)(un * (ct * hx + sg * st * nx));
        ((R *)a.dst.uy)[j] = (R)(un * (ct * hy + sg * st * ny));
        ((R *)a.dst.uz)[j] = (R)(un * (ct * hz + sg * st * nz));
        ((R *)a.dst.w)[j] = wh;
        if (chi) ((R *)a.dst.chi)[j] = (R)(sc / sw);
        const uint64_t uid = base + (uint64_t)j;
        a.dst.uid[j] = uid;
        a.dst.n_ev[j] = 0u;
        a.dst.tau[j] = initial_tau(a.seed, uid);
    }
}

hipError_t launch_merge(MergeArgs a, int prec, int mbin_passes, int cell_passes, int n_cu, hipStream_t s) {
    const int64_t cap = a.src.cap;
    const unsigned ge = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + 255) / 256, (int64_t)n_cu * 16));
    hipLaunchKernelGGL(k_merge_zero, dim3(1), dim3(64), 0, s, a.cnt);
    if (prec == 0) hipLaunchKernelGGL((k_merge_keys<double>), dim3(ge), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_merge_keys<float>), dim3(ge), dim3(256), 0, s, a);
    RadixBufs b = {{a.key[0], a.key[1]}, {a.idx[0], a.idx[1]}, a.hist, a.hoff};
    int cur = launch_radix_passes8(b, 0, a.src.count, cap, mbin_passes, n_cu, a.ws, s);
    hipLaunchKernelGGL(k_merge_rekey, dim3(ge), dim3(256), 0, s, a.g, b.idx[cur], b.key[cur], a.src.count, cap);
    cur = launch_radix_passes8(b, cur, a.src.count, cap, cell_passes, n_cu, a.ws, s);
    // sorted keys and order in (key[cur], idx[cur]); the other pair, g and o are free
    const uint32_t *kf = b.key[cur], *idx = b.idx[cur];
    uint32_t *head = b.key[cur ^ 1], *hscan = b.idx[cur ^ 1], *gstart = a.g, *ooff = a.o;
    uint32_t *osz = b.key[cur];                       // the sorted keys are dead after k_merge_heads
    hipLaunchKernelGGL(k_merge_heads, dim3(ge), dim3(256), 0, s, kf, idx, a.mkey, a.key_out, a.cnt, head);
    launch_scan_u32(head, hscan, &a.cnt[0], cap, n_cu, a.ws, s);
    hipLaunchKernelGGL(k_merge_starts, dim3(ge), dim3(256), 0, s, head, hscan, a.cnt, gstart);
    hipLaunchKernelGGL(k_merge_sizes, dim3(ge), dim3(256), 0, s, gstart, a.cnt, a.min_group, osz);
    launch_scan_u32(osz, ooff, &a.cnt[1], cap, n_cu, a.ws, s);
    hipLaunchKernelGGL(k_merge_total, dim3(1), dim3(64), 0, s, osz, ooff, a.cnt, a.uid_next, a.dst.count);
    const unsigned gw = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + 3) / 4, (int64_t)n_cu * 8));
    if (prec == 0) {
        hipLaunchKernelGGL((k_merge_copy<double>), dim3(ge), dim3(256), 0, s, a, idx, head, hscan, gstart, ooff);
        hipLaunchKernelGGL((k_merge_groups<double>), dim3(gw), dim3(256), 0, s, a, idx, gstart, ooff);
    } else {
        hipLaunchKernelGGL((k_merge_copy<float>), dim3(ge), dim3(256), 0, s, a, idx, head, hscan, gstart, ooff);
        hipLaunchKernelGGL((k_merge_groups<float>), dim3(gw), dim3(256), 0, s, a, idx, gstart, ooff);
    }
    return hipGetLastError();
}

}  // namespace qed
