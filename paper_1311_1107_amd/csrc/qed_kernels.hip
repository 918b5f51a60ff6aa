// qed_kernels.hip -- gfx950 kernels of the per-particle radiation and QED step
// (Lobet et al., arXiv:1311.1107, Secs. 2-3).
//
// The particle kernels are persistent: a fixed grid of workgroups walks tiles
// of consecutive particles, each XCD taking a contiguous range of tiles.
// Particles are structure-of-arrays; each tile reads and writes its particles
// once with coalesced accesses.  A step that creates particles runs in three
// passes: the physics pass advances every particle and records per-tile
// append counts (and, for emissions, a staged record per emitting particle),
// a scan pass forms the prefixes over tiles with a decoupled look-back, and an
// append pass writes the new particles at tile prefix + in-tile rank, which
// reproduces the serial order of the parents.  The in-place compaction keeps
// the single-pass ticketed look-back.
#include "qed_kernels.h"

#include <climits>

namespace qed {

// ------------------------------------------------------------------------
// fields
// ------------------------------------------------------------------------
// Plane wave from a_y = a0 sin^2(pi phi/Phi) sin(phi), phi = t - x:
// E_y = B_z = -(da_y/dphi).
// inv_Phi = 1/Phi is given, so that no lane divides.
template <typename R>
__device__ __forceinline__ R plane_wave_da(double t, R x, double a0, double Phi, double inv_Phi);

template <>
__device__ __forceinline__ double plane_wave_da<double>(double t, double x, double a0, double Phi, double inv_Phi) {
    const double phi = t - x;
    if (!(phi > 0.0 && phi < Phi)) return 0.0;
    const double k = kPi * inv_Phi;                    // envelope wave number pi/Phi
    double se, ce, sp, cp;
    sincos(k * phi, &se, &ce);
    sincos(phi, &sp, &cp);
    return a0 * (k * (2.0 * se * ce) * sp + se * se * cp);
}

template <>
__device__ __forceinline__ float plane_wave_da<float>(double t, float x, double a0, double Phi, double inv_Phi) {
    // phases formed and reduced in FP64, in revolutions: the envelope's
    // phi/(2 Phi) in [0, 1/2) and the carrier's phi/(2 pi) less its nearest
    // integer; their sines and cosines from the hardware's single-precision
    // V_SIN_F32 / V_COS_F32 (arguments in revolutions)
    const double phi = t - (double)x;
    if (!(phi > 0.0 && phi < Phi)) return 0.0f;
    const double rc = phi * (0.5 / kPi);
    const float re = (float)(phi * (0.5 * inv_Phi));
    const float rr = (float)(rc - rint(rc));
    const float se = __builtin_amdgcn_sinf(re), ce = __builtin_amdgcn_cosf(re);
    const float sp = __builtin_amdgcn_sinf(rr), cp = __builtin_amdgcn_cosf(rr);
    return (float)a0 * ((float)(kPi * inv_Phi) * (2.0f * se * ce) * sp + se * se * cp);
}

// Quadratic (TSC) weights for offset d from the nearest node.
template <typename R>
__device__ __forceinline__ void tsc_w(R d, R w[3]) {
    w[0] = R(0.5) * (R(0.5) - d) * (R(0.5) - d);
    w[1] = fma(-d, d, R(0.75));
    w[2] = R(0.5) * (R(0.5) + d) * (R(0.5) + d);
}

// Quadratic (TSC) weights about the nearest node.
template <typename R>
__device__ __forceinline__ int64_t tsc(R g, R w[3]) {
    // far outside the grid (or NaN): a node index that every bounds test rejects
    if (!(g > R(-1.0e6) && g < R(1.0e6))) g = R(-1.0e6);
    const R f = floor(g + R(0.5));
    tsc_w<R>(g - f, w);
    return (int64_t)f;
}

// Sum of w_x[a] w_y[b] w_z[c] v[a][b][c], contracted one axis at a time
// (z rows, then y, then x) in one fixed order with explicit FMAs, so that the
// direct and the LDS-staged gathers give the same bits for the same node
// values.
template <typename R>
__device__ __forceinline__ R tsc_sum(const R wx[3], const R wy[3], const R wz[3], const float v[27]) {
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R plane = R(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const float *r = v + 9 * a + 3 * b;
            R row = wz[0] * (R)r[0];
            row = fma(wz[1], (R)r[1], row);
            row = fma(wz[2], (R)r[2], row);
            plane = b == 0 ? wy[0] * row : fma(wy[b], row, plane);
        }
        acc = a == 0 ? wx[0] * plane : fma(wx[a], plane, acc);
    }
    return acc;
}

// Stencils of one particle: along each axis the first node and the offset
// from the nearest node, for components on integer nodes ([0]) and on
// half-integer nodes ([1]); the weights are formed where they are used.
template <typename R>
struct Stencil {
    int s[3][2];
    R d[3][2];
};

template <typename R>
__device__ __forceinline__ void make_stencil(const FieldDev &f, R x, R y, R z, Stencil<R> &st) {
    const R g[3] = {(x - (R)f.x0) * (R)f.inv_dx, (y - (R)f.y0) * (R)f.inv_dy, (z - (R)f.z0) * (R)f.inv_dz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            R gg = h ? g[d] - R(0.5) : g[d];
            // far outside the grid (or NaN): a node index that every bounds test rejects
            if (!(gg > R(-1.0e6) && gg < R(1.0e6))) gg = R(-1.0e6);
            const R fl = floor(gg + R(0.5));
            st.d[d][h] = gg - fl;
            st.s[d][h] = (int)fl - 1;
        }
    }
}


// Yee staggering of Ex Ey Ez Bx By Bz along x, y, z: 1 = half a cell off.
constexpr int kHalf[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

__constant__ double kYeeStag[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

template <typename R>
__device__ __forceinline__ void yee_gather(const FieldDev &f, R x, R y, R z, R E[3], R B[3]) {
    const int64_t nx = f.nx, ny = f.ny, nz = f.nz, plane = ny * nz, ncell = nx * plane;
    const R gx = (x - (R)f.x0) * (R)f.inv_dx, gy = (y - (R)f.y0) * (R)f.inv_dy, gz = (z - (R)f.z0) * (R)f.inv_dz;
    R out[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        R wx[3], wy[3], wz[3];
        const int64_t i0 = tsc<R>(gx - (R)kYeeStag[c][0], wx) - 1;
        const int64_t j0 = tsc<R>(gy - (R)kYeeStag[c][1], wy) - 1;
        const int64_t k0 = tsc<R>(gz - (R)kYeeStag[c][2], wz) - 1;
        const float *g = f.grid + c * ncell;
        // the operations of tsc_sum, in its order, with each row loaded where it is used
        R acc = R(0);
        if (i0 >= 0 && i0 + 2 < nx && j0 >= 0 && j0 + 2 < ny && k0 >= 0 && k0 + 2 < nz) {
            const float *p = g + (i0 * ny + j0) * nz + k0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R plane = R(0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const float *r = p + (a * ny + b) * nz;
                    R row = wz[0] * (R)r[0];
                    row = fma(wz[1], (R)r[1], row);
                    row = fma(wz[2], (R)r[2], row);
                    plane = b == 0 ? wy[0] * row : fma(wy[b], row, plane);
                }
                acc = a == 0 ? wx[0] * plane : fma(wx[a], plane, acc);
            }
        } else {
            // nodes outside the grid count as zero, in the same order of operations
            for (int a = 0; a < 3; ++a) {
                R plane = R(0);
                for (int b = 0; b < 3; ++b) {
                    const int64_t i = i0 + a, j = j0 + b;
                    const bool row_in = i >= 0 && i < nx && j >= 0 && j < ny;
                    float r[3];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        const int64_t k = k0 + cc;
                        r[cc] = row_in && k >= 0 && k < nz ? g[(i * ny + j) * nz + k] : 0.0f;
                    }
                    R row = wz[0] * (R)r[0];
                    row = fma(wz[1], (R)r[1], row);
                    row = fma(wz[2], (R)r[2], row);
                    plane = b == 0 ? wy[0] * row : fma(wy[b], row, plane);
                }
                acc = a == 0 ? wx[0] * plane : fma(wx[a], plane, acc);
            }
        }
        out[c] = acc;
    }
    E[0] = out[0]; E[1] = out[1]; E[2] = out[2];
    B[0] = out[3]; B[1] = out[4]; B[2] = out[5];
}

// ------------------------------------------------------------------------
// Wave-cooperative gather through LDS.  A direct gather moves 162 dwords per
// lane through the texture data path, which bounds a cell-ordered photon
// step.  Here a wave whose stencils all fall in a box of kWB nodes (6 along
// x, where photons drift, and 5 along y and z) loads the six components of
// that box into its own LDS region once (about 14 dwords per lane) and every
// lane reads its 3x3x3 stencils there at fixed strides.  Other waves gather
// directly.  Both paths sum with tsc_sum over the same node values, so the
// path taken never changes a result.  No block barrier: each wave owns its
// region.
// ------------------------------------------------------------------------
constexpr int kWBX = 6, kWBY = 5, kWBZ = 5;
constexpr int kWBVol = kWBX * kWBY * kWBZ;
constexpr int kWBFloats = 6 * kWBVol;

// Minimum over the wave, on every lane: row minima through DPP (quad
// permutations, row rotations), then the four rows.  The wave must be fully
// active.
__device__ __forceinline__ int wave_min_i32(int v) {
    auto mn = [](int a, int b) { return a < b ? a : b; };
    v = mn(v, __builtin_amdgcn_mov_dpp(v, 0xb1, 0xf, 0xf, false));     // quad_perm 1,0,3,2
    v = mn(v, __builtin_amdgcn_mov_dpp(v, 0x4e, 0xf, 0xf, false));     // quad_perm 2,3,0,1
    v = mn(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xf, 0xf, false));    // row_ror 4
    v = mn(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, false));    // row_ror 8
    return mn(mn(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
              mn(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Called by all lanes of the wave; act marks lanes that need the field.
// after_loads() runs once, as soon as the gather's own grid loads have been
// consumed: memory operations it issues are not waited for by the gather.
template <typename R, typename AfterLoads>
__device__ __forceinline__ void yee_gather_wave(const FieldDev &f, bool act, R x, R y, R z, R E[3], R B[3],
                                                float *box, AfterLoads &&after_loads) {
    const int64_t nx = f.nx, ny = f.ny, nz = f.nz, ncell = nx * ny * nz;
    Stencil<R> st;
    make_stencil<R>(f, x, y, z, st);
    const int64_t nn[3] = {nx, ny, nz};
    int lo[3], hi[3];
    bool near = act;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int s0 = st.s[d][0], s1 = st.s[d][1];
        lo[d] = s0 < s1 ? s0 : s1;
        hi[d] = (s0 > s1 ? s0 : s1) + 2;
        near = near && hi[d] >= 0 && (int64_t)lo[d] < nn[d];
    }
    const uint64_t m_near = __ballot(near);
    if (m_near == 0ull) {                                   // the whole wave sees a zero field
        E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = R(0);
        after_loads();
        return;
    }
    int o[3], ext[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[d] = wave_min_i32(near ? lo[d] : INT_MAX);
        ext[d] = -wave_min_i32(near ? -hi[d] : INT_MAX) - o[d] + 1;    // nodes spanned along d
    }
    if (ext[0] > kWBX || ext[1] > kWBY || ext[2] > kWBZ) {
        if (near) yee_gather<R>(f, x, y, z, E, B);
        else E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = R(0);
        after_loads();
        return;
    }
    // stage the box: node e = (p kWBY + q) kWBZ + r; every load of the lane is
    // issued before the first LDS write
    constexpr int kU = (kWBVol + kWave - 1) / kWave;
    bool span[kU], in[kU];
    int64_t off[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int e = lane_id() + u * kWave;
        const int p = e / (kWBY * kWBZ), q = (e / kWBZ) % kWBY, r = e % kWBZ;
        // only the nodes the wave's stencils span are stored (the rest are never read)
        span[u] = e < kWBVol && p < ext[0] && q < ext[1] && r < ext[2];
        const int64_t i = o[0] + p, j = o[1] + q, k = o[2] + r;
        in[u] = span[u] && i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
        off[u] = in[u] ? (i * ny + j) * nz + k : 0;
    }
    float v[kU][6];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[u][c] = in[u] ? f.grid[c * ncell + off[u]] : 0.0f;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int e = lane_id() + u * kWave;
        if (span[u]) {
#pragma unroll
            for (int c = 0; c < 6; ++c) box[c * kWBVol + e] = v[u][c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    after_loads();
    R out[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int hx = kHalf[c][0], hy = kHalf[c][1], hz = kHalf[c][2];
        const int base = near ? ((st.s[0][hx] - o[0]) * kWBY + (st.s[1][hy] - o[1])) * kWBZ + (st.s[2][hz] - o[2]) : 0;
        const float *p = box + c * kWBVol + base;
        float v[27];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) v[9 * a + 3 * b + cc] = p[(a * kWBY + b) * kWBZ + cc];
        R wx[3], wy[3], wz[3];
        tsc_w<R>(st.d[0][hx], wx);
        tsc_w<R>(st.d[1][hy], wy);
        tsc_w<R>(st.d[2][hz], wz);
        out[c] = near ? tsc_sum<R>(wx, wy, wz, v) : R(0);
    }
    // the box is rewritten only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    E[0] = out[0]; E[1] = out[1]; E[2] = out[2];
    B[0] = out[3]; B[1] = out[4]; B[2] = out[5];
}

template <typename R, int FK>
__device__ __forceinline__ void field_at(const FieldDev &f, double t, R x, R y, R z,
                                         double a0, double Phi, double inv_Phi, R E[3], R B[3]) {
    if (FK == FIELD_UNIFORM) {
        E[0] = (R)f.E[0]; E[1] = (R)f.E[1]; E[2] = (R)f.E[2];
        B[0] = (R)f.B[0]; B[1] = (R)f.B[1]; B[2] = (R)f.B[2];
    } else if (FK == FIELD_PLANE || FK == FIELD_BUNCHED || FK == FIELD_BUNCHED_GLOBAL) {
        const R da = plane_wave_da<R>(t, x, a0, Phi, inv_Phi);
        E[0] = R(0); E[1] = -da; E[2] = R(0);
        B[0] = R(0); B[1] = R(0); B[2] = -da;
    } else {
        yee_gather<R>(f, x, y, z, E, B);
    }
}

// ------------------------------------------------------------------------
// helpers for the per-tile epilogue
// ------------------------------------------------------------------------
__device__ __forceinline__ void status_flag(unsigned long long *st, unsigned long long bit) {
    atomicOr(st + 0, bit);
}
__device__ __forceinline__ void status_need(unsigned long long *st, int which, int64_t v) {
    atomicMax(st + 1 + which, (unsigned long long)v);
}

// Energy sums of one wave's tile into its tally slot, added with an FP64
// atomic that returns nothing (the wave does not wait for it).  With a slot
// per tile each slot takes one addition per launch, so the sums do not depend
// on the schedule; with fewer slots, their order does.
template <int NE>
__device__ __forceinline__ void wave_energy(const TallyDev &tal, int64_t tile, double (&e)[NE]) {
    static_assert(NE % 2 == 0, "energies are summed in pairs");
    // a tally sized for the launch has a slot per tile: no division then
    const int64_t sl = tile < tal.n_slots ? tile : tile % tal.n_slots;
#pragma unroll
    for (int k = 0; k < NE; k += 2) {
        if (__ballot(e[k] != 0.0 || e[k + 1] != 0.0) == 0ull) continue;
        double s0, s1;
        wave_sum2_f64_dpp(e[k], e[k + 1], s0, s1);
        if (lane_id() == 0) {
            if (s0 != 0.0) unsafeAtomicAdd(tal.energy + sl * kNEnergy + k, s0);
            if (s1 != 0.0) unsafeAtomicAdd(tal.energy + sl * kNEnergy + k + 1, s1);
        }
    }
}

// Add the block's integer counts into the tally (commutative, so exact).
__device__ __forceinline__ void block_counts(const TallyDev &tal, int (&c)[N_COUNT_USED], int64_t *s_cnt) {
    if (threadIdx.x < N_COUNT_USED) s_cnt[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) {
        uint32_t v = (uint32_t)c[k];
        if (__ballot(v != 0u)) {
            v = wave_sum_u32(v);
            if (lane_id() == 0 && v) atomicAdd((unsigned long long *)&s_cnt[k], (unsigned long long)v);
        }
    }
    __syncthreads();
    if (threadIdx.x < N_COUNT_USED && s_cnt[threadIdx.x])
        atomicAdd((unsigned long long *)(tal.count + threadIdx.x), (unsigned long long)s_cnt[threadIdx.x]);
}

// ------------------------------------------------------------------------
// Physics passes walk the tiles of a launch with a persistent grid.  The tile
// range is cut into eight contiguous pieces, one per XCD (the dispatcher deals
// block ids to the eight XCDs in turn), so that each XCD's L2 serves a compact
// run of particles.  Tiles are independent here: appends are placed later by
// the scan and append passes, so no tile waits for another.
// ------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_tile(int64_t it, int64_t n_tiles, bool rev = false) {
    const int64_t g8 = gridDim.x >> 3;             // the grid is a multiple of 8
    const int64_t x = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int64_t lo = n_tiles * x / 8, hi = n_tiles * (x + 1) / 8;
    const int64_t k = l + it * g8;
    return lo + k < hi ? (rev ? hi - 1 - k : lo + k) : -1;
}

// Successive steps walk the tiles in opposite directions, so that a step
// starts on the lines that the previous one wrote last (those are still in
// the memory-side cache).  The direction follows the parity of the step
// number t / dt; results do not depend on it.
__device__ __forceinline__ bool walk_reverse(double t, double dt) {
    const int odd = dt > 0.0 && (llrint(t / dt) & 1) != 0;
    return __builtin_amdgcn_readfirstlane(odd) != 0;
}

// s_waitcnt vmcnt(0), leaving the other counters free (expcnt 7, lgkmcnt 15)
constexpr int kWaitVmem = 0x0F70;

// ------------------------------------------------------------------------
// Lepton step: Boris push, chi_e, Sokolov or optical-depth Monte Carlo.
// ------------------------------------------------------------------------
// Emissions of one particle in one step, kept in registers: slots are written
// through compile-time indices so that no scratch memory is used.
template <typename R>
struct Emitted {
    R gg[kMaxEvents];      // gamma_gamma
    R chig[kMaxEvents];    // chi_gamma at creation
    uint8_t dst[kMaxEvents];   // 0 pushed, 1 recorded, 2 tallied, 3 below threshold
    int n;
    __device__ __forceinline__ void put(int k, R g, R c, uint8_t d) {
#pragma unroll
        for (int j = 0; j < kMaxEvents; ++j)
            if (j == k) { gg[j] = g; chig[j] = c; dst[j] = d; }
        n = k + 1;
    }
};

// The address of element `first` of p in scalar registers (`first` is uniform
// over the wave): an access to element first + lane then takes a fixed 32-bit
// lane offset from it, with no 64-bit vector address arithmetic.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *wave_base(T *p, int64_t first) {
    const uint64_t v = (uint64_t)(p + first);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (__attribute__((address_space(1))) T *)((hi << 32) | lo);
}

// Bunch of each lane in the batched form (bunch b holds [offsets[b],
// offsets[b+1])): the wave counts the offsets at or below its first particle,
// 64 at a time, then each lane steps forward past the bunch ends before it.
// Called by all lanes of the wave.
__device__ __forceinline__ int lane_bunch(const int64_t *offsets, int n_bunches, int64_t first, int64_t i) {
    int b = 0;
    for (int base = 1; base <= n_bunches; base += kWave) {
        const int k = base + lane_id();
        const uint64_t m = __ballot(k <= n_bunches && offsets[k] <= first);
        b += __popcll(m);
        if (m != ~0ull) break;
    }
    while (b + 1 < n_bunches && i >= offsets[b + 1]) ++b;
    return b;
}

// Stream pass of the lepton step.  Each wave steps its own tile of 64
// particles, with no block barrier: field at x^n, Boris push to u_L, chi_e
// (Eq. 1), then either the Sokolov step (Eqs. 4-5) or, for the optical-depth
// Monte Carlo (Eqs. 6-8), the decrement of tau by W dt.  A particle whose
// tau runs out within the step is left as it was: its state after the push
// goes to an event item (slot tile * 64 + rank), and the event pass finishes
// it with the other event particles in full waves.  The tile's item count
// goes to tile_cnt0 for the scan that lists the items.
template <typename R, int FK>
__global__ void __launch_bounds__(256)
k_lepton_stream(PushArgs a) {
    __shared__ R s_lh[kMaxChiNodes];
    __shared__ R s_lg[kMaxChiNodes];
    __shared__ float s_box[FK == FIELD_YEE ? kMaxWaves * kWBFloats : 1];
    __shared__ int64_t s_cnt[N_COUNT_USED];
    extern __shared__ __align__(16) unsigned char s_dyn[];      // bunch table (batched form)

    const int tid = threadIdx.x, lane = lane_id(), nw = blockDim.x / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);    // uniform over the wave
    const TablesDev &tb = a.tab;
    for (int k = tid; k < tb.e_n_chi; k += blockDim.x) {
        s_lh[k] = (R)tb.ln_hrad[k];
        s_lg[k] = (R)tb.ln_g[k];
    }
    // batched form: offsets, amplitudes, phase lengths 2 pi n_periods and their
    // reciprocals of the bunches in LDS (FIELD_BUNCHED), or read from global
    // memory for a table too large for it (FIELD_BUNCHED_GLOBAL).  The two are
    // separate instantiations: a global load here would have to wait for the
    // next tile's loads issued before it.
    const int nb = a.f.n_bunches;
    int64_t *so = (int64_t *)s_dyn;
    double *sa = (double *)(so + nb + 1), *s_phi = sa + nb, *s_iphi = s_phi + nb;
    if (FK == FIELD_BUNCHED) {
        for (int k = tid; k <= nb; k += blockDim.x) so[k] = a.f.offsets[k];
        for (int k = tid; k < nb; k += blockDim.x) {
            sa[k] = a.f.a0s[k];
            s_phi[k] = 2.0 * kPi * a.f.nper[k];
            s_iphi[k] = 1.0 / s_phi[k];
        }
    }
    const int64_t n = *a.lep.count;
    const double t = a.st.d_step ? a.st.t + (double)(*a.st.d_step) * a.st.dt : a.st.t;
    const double dt = a.st.dt;
    const R dtr = (R)dt;
    const bool rev = walk_reverse(t, dt);
    const int64_t n_chunks = (n + blockDim.x - 1) / blockDim.x;
    const int64_t n_tiles = (n + kWave - 1) / kWave;
    const R q = (R)a.c.q, hq = R(0.5) * q * dtr;
    const R es_inv = (R)a.c.es_inv, Ah = (R)a.c.A, tau0 = (R)a.c.tau0;
    const R lnchi0 = (R)tb.e_lnchi0, inv_d = (R)tb.e_inv_dlnchi;
    R *X = (R *)a.lep.x, *Y = (R *)a.lep.y, *Z = (R *)a.lep.z;
    R *UX = (R *)a.lep.ux, *UY = (R *)a.lep.uy, *UZ = (R *)a.lep.uz;
    const R *Wt = (const R *)a.lep.w;
    ItemRec<R> *items = (ItemRec<R> *)a.ws.stage.item;
    int cnt[N_COUNT_USED];
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) cnt[k] = 0;
    __syncthreads();

    // the state of a wave's next tile is loaded before the current one is
    // stepped, which hides the HBM latency behind the arithmetic
    int64_t chunk = xcd_tile(0, n_chunks, rev);
    R n_x = R(0), n_y = R(0), n_z = R(0), n_ux = R(0), n_uy = R(0), n_uz = R(0), n_w = R(0);
    double n_tau = 0.0;
    const uint32_t ul = (uint32_t)lane;
    if (chunk >= 0 && chunk * blockDim.x + tid < n) {
        const int64_t b = (chunk * nw + wid) * kWave;
        n_x = wave_base(X, b)[ul]; n_y = wave_base(Y, b)[ul]; n_z = wave_base(Z, b)[ul];
        n_ux = wave_base(UX, b)[ul]; n_uy = wave_base(UY, b)[ul]; n_uz = wave_base(UZ, b)[ul];
        n_w = wave_base(Wt, b)[ul]; n_tau = wave_base(a.lep.tau, b)[ul];
    }
    for (int64_t it = 0; chunk >= 0; ++it) {
        const int64_t tile = chunk * nw + wid;             // = i / 64
        const int64_t i = chunk * blockDim.x + tid;
        const bool live = i < n;
        const R x = n_x, y = n_y, z = n_z, ux = n_ux, uy = n_uy, uz = n_uz, wgt_i = n_w;
        const double tau_i = n_tau;
        const int64_t next = xcd_tile(it + 1, n_chunks, rev);
        auto prefetch = [&]() {
            if (next >= 0 && next * blockDim.x + tid < n) {
                const int64_t b = (next * nw + wid) * kWave;
                n_x = wave_base(X, b)[ul]; n_y = wave_base(Y, b)[ul]; n_z = wave_base(Z, b)[ul];
                n_ux = wave_base(UX, b)[ul]; n_uy = wave_base(UY, b)[ul]; n_uz = wave_base(UZ, b)[ul];
                n_w = wave_base(Wt, b)[ul]; n_tau = wave_base(a.lep.tau, b)[ul];
            }
        };
        // with a grid the loads go out after the gather's (whose wait would include them)
        if constexpr (FK != FIELD_YEE) prefetch();
        const int64_t tile0 = tile * kWave;                 // = i - lane
        double en[kNEnergy];
#pragma unroll
        for (int k = 0; k < kNEnergy; ++k) en[k] = 0.0;
        double a0 = a.f.a0, Phi = a.f.Phi, inv_Phi = a.f.inv_Phi;
        if (FK == FIELD_BUNCHED) {
            const int b = lane_bunch(so, nb, tile * kWave, i);
            if (live) { a0 = sa[b]; Phi = s_phi[b]; inv_Phi = s_iphi[b]; }
        } else if (FK == FIELD_BUNCHED_GLOBAL) {
            const int b = lane_bunch(a.f.offsets, nb, tile * kWave, i);
            if (live) { a0 = a.f.a0s[b]; Phi = 2.0 * kPi * a.f.nper[b]; inv_Phi = 1.0 / Phi; }
        }
        R E[3], B[3];
        if constexpr (FK == FIELD_YEE) yee_gather_wave<R>(a.f, live, x, y, z, E, B, s_box + wid * kWBFloats, prefetch);
        bool event = false, put_tau = false;
        R uLx = R(0), uLy = R(0), uLz = R(0), gL = R(1), chi = R(0), W = R(0), wgt = R(0);
        R xn = R(0), yn = R(0), zn = R(0), unx = R(0), uny = R(0), unz = R(0);
        double tau = 0.0, tau_new = 0.0;
        if (live) {
            if constexpr (FK != FIELD_YEE) field_at<R, FK>(a.f, t, x, y, z, a0, Phi, inv_Phi, E, B);
            const R g_old = Math<R>::sqrt_(R(1) + (ux * ux + uy * uy + uz * uz));

            // Boris: half electric kick, magnetic rotation, half kick
            const R umx = ux + hq * E[0], umy = uy + hq * E[1], umz = uz + hq * E[2];
            const R gm = Math<R>::sqrt_(R(1) + (umx * umx + umy * umy + umz * umz));
            const R hg = Math<R>::div_(hq, gm);
            const R tx = hg * B[0], ty = hg * B[1], tz = hg * B[2];
            const R t2 = tx * tx + ty * ty + tz * tz;
            const R s2 = R(2) * Math<R>::rcp_(R(1) + t2);
            const R sx = s2 * tx, sy = s2 * ty, sz = s2 * tz;
            const R px = umx + (umy * tz - umz * ty);
            const R py = umy + (umz * tx - umx * tz);
            const R pz = umz + (umx * ty - umy * tx);
            const R qx = umx + (py * sz - pz * sy);
            const R qy = umy + (pz * sx - px * sz);
            const R qz = umz + (px * sy - py * sx);
            uLx = qx + hq * E[0]; uLy = qy + hq * E[1]; uLz = qz + hq * E[2];
            gL = Math<R>::sqrt_(R(1) + (uLx * uLx + uLy * uLy + uLz * uLz));
            wgt = wgt_i;
            en[E_WORK] = (double)wgt * (double)(gL - g_old);

            chi = chi_of<R>(es_inv, gL, uLx, uLy, uLz, E, B);
            unx = uLx; uny = uLy; unz = uLz;
            R dvx = R(0), dvy = R(0), dvz = R(0);
            int rad = a.st.rad;
            if (!__builtin_isfinite(chi) || !__builtin_isfinite(gL)) { cnt[C_NAN]++; rad = RAD_NONE; status_flag(a.ws.status, 2ull); }

            if (rad == RAD_SOKOLOV || (rad == RAD_HYBRID && (double)chi < a.st.chi_switch)) {
                // Sokolov scheme (Eq. 4) with P_rad of Eq. 5
                cnt[C_SOKOLOV]++;
                const R igL = Math<R>::rcp_(gL);
                const R vx = uLx * igL, vy = uLy * igL, vz = uLz * igL;
                const R fx = q * (E[0] + (vy * B[2] - vz * B[1]));
                const R fy = q * (E[1] + (vz * B[0] - vx * B[2]));
                const R fz = q * (E[2] + (vx * B[1] - vy * B[0]));
                const R vf = vx * fx + vy * fy + vz * fz;
                const R g = chi > R(0) ? g_at<R>(s_lg, tb, lnchi0, inv_d, chi) : R(1);
                // variant: delta_v with the quantum-reduced tau_0 g(chi)
                const R tq = (a.st.variants & VAR_SOKOLOV_G) ? tau0 * g : tau0;
                const R tden = Math<R>::div_(tq, R(1) + tq * vf);
                dvx = tden * (fx - vx * vf);
                dvy = tden * (fy - vy * vf);
                dvz = tden * (fz - vz * vf);
                const R P = (R(2) / R(3)) * Ah * chi * chi * g;
                const R bx = dvy * B[2] - dvz * B[1], by = dvz * B[0] - dvx * B[2], bz = dvx * B[1] - dvy * B[0];
                const R Pg = P * igL;
                unx = uLx + dtr * (q * bx - Pg * uLx);
                uny = uLy + dtr * (q * by - Pg * uLy);
                unz = uLz + dtr * (q * bz - Pg * uLz);
                en[E_RAD] = (double)wgt * (double)P * dt;
            } else if (rad == RAD_MC || rad == RAD_HYBRID) {
                // optical-depth Monte Carlo, Eqs. 6-8: dtau/dt = W
                cnt[C_MC]++;
                const R p = Math<R>::sqrt_(uLx * uLx + uLy * uLy + uLz * uLz);
                if (p > R(0) && chi > R(0)) {
                    bool above = false;
                    W = Math<R>::div_(Ah * h_rad_at<R>(s_lh, tb, lnchi0, inv_d, chi, above), gL);
                    if (above) cnt[C_RANGE]++;
                }
                tau = tau_i;
                const double Wd = (double)W;
                if (!(W > R(0)) || tau > Wd * dt) { put_tau = true; tau_new = tau - Wd * dt; }
                else event = true;                          // finished by the event pass
            }
            if (!event) {
                const R gn = Math<R>::sqrt_(R(1) + (unx * unx + uny * uny + unz * unz));
                const R ign = Math<R>::rcp_(gn);
                xn = x + dtr * (unx * ign + dvx);
                yn = y + dtr * (uny * ign + dvy);
                zn = z + dtr * (unz * ign + dvz);
            }
        }
        // The next tile's loads went out before the arithmetic above.  Wait for
        // them here, before this tile's stores: the memory counter retires in
        // issue order, so a wait placed after the stores (where the loaded
        // registers are next read) would wait for the stores as well.
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        if (put_tau) wave_base(a.lep.tau, tile0)[ul] = tau_new;
        if (live && !event) {
            wave_base(X, tile0)[ul] = xn; wave_base(Y, tile0)[ul] = yn; wave_base(Z, tile0)[ul] = zn;
            wave_base(UX, tile0)[ul] = unx; wave_base(UY, tile0)[ul] = uny; wave_base(UZ, tile0)[ul] = unz;
        }
        uint32_t n_items;
        const uint32_t rank = ballot_excl(event, n_items);
        if (event) {
            const ItemRec<R> r = {{x, y, z, uLx, uLy, uLz, E[0], E[1], E[2], B[0], B[1], B[2], gL, chi, W, wgt},
                                  tau, (uint32_t)i, 0u};
            items[tile * kWave + rank] = r;
        }
        if (tile < n_tiles) {
            if (lane == 0) a.ws.tile_cnt0[tile] = n_items;
            wave_energy<kNEnergy>(a.tal, tile, en);
        }
        chunk = next;
    }
    block_counts(a.tal, cnt, s_cnt);
}

// Event pass of the lepton step.  Each wave takes 64 consecutive event items
// (in particle order) and runs their emissions in full waves: the local-time
// sub-loop of at most kmax events, each a Philox draw, the photon fraction
// from the inverse CDF of Eq. 7 and the recoil of Eq. 8, the new chi_e and W
// after it; then the particle's new momentum, position, tau and event
// counter.  Photons to be stored go to an emission record at the item's
// dense position; the counts of each 64-item chunk go to tile_cnt0/1 for the
// scan of the appends.  kSpline: the quantile table is read through the
// spline (a separate instantiation, so that the bilinear form keeps its
// registers).
template <typename R, bool kSpline>
__global__ void __launch_bounds__(256)
k_lepton_events(PushArgs a) {
    __shared__ R s_lh[kMaxChiNodes];
    __shared__ int64_t s_cnt[N_COUNT_USED];

    const int tid = threadIdx.x, lane = lane_id(), nw = blockDim.x / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);    // uniform over the wave
    const TablesDev &tb = a.tab;
    for (int k = tid; k < tb.e_n_chi; k += blockDim.x) s_lh[k] = (R)tb.ln_hrad[k];
    const int64_t n_items = a.ws.info->n_items;
    const int64_t n_chunks = (n_items + kWave - 1) / kWave;
    const double dt = a.st.dt;
    const R dtr = (R)dt;
    const R es_inv = (R)a.c.es_inv, Ah = (R)a.c.A;
    const R lnchi0 = (R)tb.e_lnchi0, inv_d = (R)tb.e_inv_dlnchi;
    const R *qtab = emit_q_ptr<R>(tb), *qspl = kSpline ? emit_qs_ptr<R>(tb) : nullptr;
    R *X = (R *)a.lep.x, *Y = (R *)a.lep.y, *Z = (R *)a.lep.z;
    R *UX = (R *)a.lep.ux, *UY = (R *)a.lep.uy, *UZ = (R *)a.lep.uz;
    const ItemRec<R> *items = (const ItemRec<R> *)a.ws.stage.item;
    R *rec = (R *)a.ws.stage.rec;
    const int64_t slots = a.ws.stage.slots;
    int cnt[N_COUNT_USED];
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) cnt[k] = 0;
    __syncthreads();

    const int64_t waves = (int64_t)gridDim.x * nw;
    // the streaming pass wrote the far end of its walk last: start there
    const double t_ev = a.st.d_step ? a.st.t + (double)(*a.st.d_step) * a.st.dt : a.st.t;
    const bool fwd = walk_reverse(t_ev, a.st.dt);
    for (int64_t w = (int64_t)blockIdx.x * nw + wid; w < n_chunks; w += waves) {
        const int64_t c = fwd ? w : n_chunks - 1 - w;
        const int64_t d = c * kWave + lane;
        const bool have = d < n_items;
        double en[kNEnergy];
#pragma unroll
        for (int k = 0; k < kNEnergy; ++k) en[k] = 0.0;
        Emitted<R> em;
        em.n = 0;
        R x = R(0), y = R(0), z = R(0), uhx = R(0), uhy = R(0), uhz = R(0), wgt = R(0);
        if (have) {
            const ItemRec<R> r = items[a.ws.stage.item_map[d]];
            const int64_t i = r.idx;
            uint32_t nev = a.lep.n_ev[i];
            const uint64_t uid = a.lep.uid[i];
            const R *v = r.v;
            x = v[0]; y = v[1]; z = v[2];
            const R uLx = v[3], uLy = v[4], uLz = v[5];
            const R E[3] = {v[6], v[7], v[8]}, B[3] = {v[9], v[10], v[11]};
            R gam = v[12], ce = v[13], W = v[14];
            wgt = v[15];
            double tau = r.tau;
            R p = Math<R>::sqrt_(uLx * uLx + uLy * uLy + uLz * uLz);
            if (p > R(0)) { const R ip = Math<R>::rcp_(p); uhx = uLx * ip; uhy = uLy * ip; uhz = uLz * ip; }
            double t_left = dt;
            int k = 0;
            for (;;) {
                const double Wd = (double)W;
                if (!(W > R(0)) || tau > Wd * t_left) { tau -= Wd * t_left; break; }
                if (k == a.st.kmax) { tau -= Wd * t_left; cnt[C_CAP]++; break; }
                t_left -= (tau > 0.0 ? tau : 0.0) / Wd;
                const U64x4 o = philox4x64_10(uid, (uint64_t)nev, (uint64_t)RNG_EMIT, 0ull, a.st.seed, 0ull);
                const double r1 = u01(o.a), r2 = u01(o.b);
                R xi = Math<R>::exp_(quantile<R>(qtab, qspl, (R)tb.e_ht26, (R)tb.e_hc26, tb.e_n_chi, tb.e_n_q,
                                                 lnchi0, inv_d, tb.e_logit_max, tb.e_inv_dt, Math<R>::log_(ce), r1));
                if (xi > R(1)) xi = R(1);
                const R gg = xi * gam;
                cnt[C_EMIT]++;
                uint8_t dst;
                R chig_k = R(0);
                const double eg = (double)wgt * (double)gg;
                if ((double)gg > a.st.gmin) {
                    chig_k = xi * ce;
                    if (a.pp.present && (double)chig_k > a.st.chi_push_min) { dst = 0; cnt[C_PUSH]++; en[E_PUSH] += eg; }
                    else if (a.pr.present) { dst = 1; cnt[C_REC]++; en[E_REC] += eg; }
                    else { dst = 2; cnt[C_DROP]++; en[E_DROP] += eg; }
                } else {
                    dst = 3; cnt[C_SUB]++; en[E_SUB] += eg;
                }
                em.put(k, gg, chig_k, dst);
                if (!a.st.no_recoil) {
                    // Eq. 8: |p_f| = |p| - eps_gamma/c, clamped at zero
                    p = p - gg;
                    if (p < R(0)) p = R(0);
                    gam = Math<R>::sqrt_(R(1) + p * p);
                    ce = chi_of<R>(es_inv, gam, p * uhx, p * uhy, p * uhz, E, B);
                    W = R(0);
                    if (p > R(0) && ce > R(0)) {
                        bool above = false;
                        W = Math<R>::div_(Ah * h_rad_at<R>(s_lh, tb, lnchi0, inv_d, ce, above), gam);
                        if (above) cnt[C_RANGE]++;
                    }
                }
                tau = -log(r2);
                ++nev;
                ++k;
            }
            const R unx = p * uhx, uny = p * uhy, unz = p * uhz;
            const R gn = Math<R>::sqrt_(R(1) + (unx * unx + uny * uny + unz * unz));
            const R ign = Math<R>::rcp_(gn);
            X[i] = x + dtr * (unx * ign);
            Y[i] = y + dtr * (uny * ign);
            Z[i] = z + dtr * (unz * ign);
            UX[i] = unx; UY[i] = uny; UZ[i] = unz;
            a.lep.n_ev[i] = nev;
            a.lep.tau[i] = tau;
        }
        // --- the item's emission record and the chunk's append counts -------
        uint32_t c0 = 0, c1 = 0, meta = (uint32_t)em.n;
#pragma unroll
        for (int k = 0; k < kMaxEvents; ++k)
            if (k < em.n) {
                c0 += em.dst[k] == 0;
                c1 += em.dst[k] == 1;
                meta |= (uint32_t)em.dst[k] << (3 + 2 * k);
            }
        if (have) {
            if (c0 + c1 > 0) {
                rec[0 * slots + d] = x; rec[1 * slots + d] = y; rec[2 * slots + d] = z;
                rec[3 * slots + d] = uhx; rec[4 * slots + d] = uhy; rec[5 * slots + d] = uhz;
                rec[6 * slots + d] = wgt;
#pragma unroll
                for (int k = 0; k < kMaxEvents; ++k)
                    if (k < em.n) { rec[(7 + k) * slots + d] = em.gg[k]; rec[(11 + k) * slots + d] = em.chig[k]; }
            }
            a.ws.stage.meta[d] = meta;
        }
        const uint32_t t0 = wave_sum_u32(c0), t1 = wave_sum_u32(c1);
        if (lane == 0) {
            a.ws.tile_cnt0[c] = t0;
            a.ws.tile_cnt1[c] = t1;
            a.ws.stage.n_rec[c] = (uint32_t)(n_items - c * kWave < kWave ? n_items - c * kWave : kWave);
        }
        wave_energy<kNEnergy>(a.tal, c, en);
    }
    block_counts(a.tal, cnt, s_cnt);
}

// ------------------------------------------------------------------------
// Scan pass: exclusive prefixes of the physics pass's per-tile append counts
// (decoupled look-back over blocks of kScanItems x 256 counts, taken in ticket
// order).  The launch's final requester records the destination buffers'
// counts and the first id for the append pass, then advances them.
// ------------------------------------------------------------------------
constexpr int kScanItems = 16;

__global__ void __launch_bounds__(256)
k_scan_tiles(ScanArgs a) {
    __shared__ uint64_t s_ticket;
    __shared__ uint32_t s_wave[2 * kMaxWaves];
    __shared__ uint32_t s_pref[2];
    const int tid = threadIdx.x;
    const int64_t n = *a.src_count;
    const int64_t n_tiles = (n + a.tile_sz - 1) / a.tile_sz;
    const int64_t per = (int64_t)blockDim.x * kScanItems;
    const int64_t n_st = (n_tiles + per - 1) / per;
    const int64_t base0 = a.d0.present ? *a.d0.count : 0;
    const int64_t base1 = a.d1.present ? *a.d1.count : 0;
    // the item list (mode 2) hands out no ids and has no id counter
    const uint64_t uid0 = a.mode == 2 ? 0ull : *a.uid_next;
    __syncthreads();
    for (;;) {
        if (tid == 0) s_ticket = atomicAdd((unsigned long long *)a.ws.ticket, 1ull);
        __syncthreads();
        const uint64_t tk = s_ticket;
        const uint32_t epoch = (uint32_t)(tk >> 32);
        const int64_t st = (int64_t)(tk & 0xffffffffull);
        if (st >= n_st) {
            if (tid == 0 && st == n_st + (int64_t)gridDim.x - 1) {
                uint32_t t0 = 0, t1 = 0;
                if (n_st > 0) lb_wait_inclusive(a.ws.lb, n_st - 1, epoch, t0, t1);
                if (a.mode == 2) {
                    a.ws.info->n_items = (int64_t)t0;
                } else {
                    a.ws.info->base0 = base0;
                    a.ws.info->base1 = base1;
                    a.ws.info->uid0 = uid0;
                }
                if (a.mode == 2) {
                    // the item list needs no destination counts or ids
                } else if (a.mode == 0) {
                    if (a.d0.present) {
                        int64_t want = base0 + (int64_t)t0;
                        if (want > a.d0.cap) { status_flag(a.ws.status, 1ull); status_need(a.ws.status, 0, want); want = a.d0.cap; }
                        *a.d0.count = want;
                    }
                    if (a.d1.present) {
                        int64_t want = base1 + (int64_t)t1;
                        if (want > a.d1.cap) { status_flag(a.ws.status, 1ull); status_need(a.ws.status, 1, want); want = a.d1.cap; }
                        *a.d1.count = want;
                    }
                    *a.uid_next = uid0 + (uint64_t)t0 + (uint64_t)t1;
                } else {
                    int64_t we = base0 + (int64_t)t0, wp = base1 + (int64_t)t0;
                    if (we > a.d0.cap) { status_flag(a.ws.status, 1ull); status_need(a.ws.status, 2, we); we = a.d0.cap; }
                    if (wp > a.d1.cap) { status_flag(a.ws.status, 1ull); status_need(a.ws.status, 3, wp); wp = a.d1.cap; }
                    *a.d0.count = we;
                    *a.d1.count = wp;
                    *a.uid_next = uid0 + 2ull * (uint64_t)t0;
                }
                atomicAdd((unsigned long long *)a.ws.ticket,
                          (1ull << 32) - (unsigned long long)(n_st + (int64_t)gridDim.x));
            }
            break;
        }
        const int64_t b = st * per + (int64_t)tid * kScanItems;
        uint32_t v0[kScanItems], v1[kScanItems];
        uint32_t s0 = 0, s1 = 0;
        const bool whole = b + kScanItems <= n_tiles;
        if (whole) {
            // a thread's 16 counts are 64 contiguous bytes (the per-tile arrays start 64-byte
            // aligned): four 16-byte loads instead of sixteen strided ones
            const uint4 *p0 = (const uint4 *)(a.ws.tile_cnt0 + b), *p1 = (const uint4 *)(a.ws.tile_cnt1 + b);
#pragma unroll
            for (int q = 0; q < kScanItems / 4; ++q) {
                const uint4 c0 = p0[q];
                v0[4 * q] = c0.x; v0[4 * q + 1] = c0.y; v0[4 * q + 2] = c0.z; v0[4 * q + 3] = c0.w;
                if (a.mode != 2) {
                    const uint4 c1 = p1[q];
                    v1[4 * q] = c1.x; v1[4 * q + 1] = c1.y; v1[4 * q + 2] = c1.z; v1[4 * q + 3] = c1.w;
                } else {
                    v1[4 * q] = v1[4 * q + 1] = v1[4 * q + 2] = v1[4 * q + 3] = 0u;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < kScanItems; ++j) {
                const int64_t idx = b + j;
                v0[j] = idx < n_tiles ? a.ws.tile_cnt0[idx] : 0u;
                v1[j] = idx < n_tiles && a.mode != 2 ? a.ws.tile_cnt1[idx] : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            s0 += v0[j];
            s1 += v1[j];
        }
        uint32_t e0, e1, tot0, tot1;
        block_scan2(s0, s1, e0, e1, tot0, tot1, s_wave);
        if (tid < kWave) {
            uint32_t p0, p1;
            lookback2(a.ws.lb, st, epoch, tot0, tot1, p0, p1);
            if (tid == 0) { s_pref[0] = p0; s_pref[1] = p1; }
        }
        __syncthreads();
        uint32_t r0 = s_pref[0] + e0, r1 = s_pref[1] + e1;
        uint32_t q0[kScanItems], q1[kScanItems];
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t idx = b + j;
            q0[j] = r0;
            q1[j] = r1;
            // mode 2: item r0 + m of the list is the tile's m-th, at slot idx * tile_sz + m
            if (a.mode == 2 && idx < n_tiles)
                for (uint32_t m = 0; m < v0[j]; ++m)
                    a.ws.stage.item_map[r0 + m] = (uint32_t)(idx * a.tile_sz + m);
            r0 += v0[j];
            r1 += v1[j];
        }
        if (whole) {
            uint4 *p0 = (uint4 *)(a.ws.tile_pre0 + b), *p1 = (uint4 *)(a.ws.tile_pre1 + b);
#pragma unroll
            for (int q = 0; q < kScanItems / 4; ++q) {
                p0[q] = make_uint4(q0[4 * q], q0[4 * q + 1], q0[4 * q + 2], q0[4 * q + 3]);
                p1[q] = make_uint4(q1[4 * q], q1[4 * q + 1], q1[4 * q + 2], q1[4 * q + 3]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kScanItems; ++j)
                if (b + j < n_tiles) { a.ws.tile_pre0[b + j] = q0[j]; a.ws.tile_pre1[b + j] = q1[j]; }
        }
        __syncthreads();
    }
}

// Lists, in LDS, the tiles of chunk c (blockDim tiles) whose count is non-zero;
// returns how many.
__device__ __forceinline__ uint32_t list_tiles(const uint32_t *cnt, int64_t c, int64_t n_tiles,
                                               uint32_t *s_list, uint32_t *s_wave) {
    const int64_t t = c * blockDim.x + threadIdx.x;
    const bool nz = t < n_tiles && cnt[t] != 0u;
    uint32_t pos, m;
    block_scan_flag(nz, pos, m, s_wave);
    if (nz) s_list[pos] = threadIdx.x;
    __syncthreads();
    return m;
}

// Append pass of the lepton step: photons from the emission records of the
// event pass (chunks of 64 items), at the offsets of the scan pass, with ids
// in the parents' serial order.
template <typename R>
__global__ void __launch_bounds__(256)
k_push_append(PushArgs a) {
    __shared__ int64_t s_cnt[N_COUNT_USED];
    const int64_t n = a.ws.info->n_items;
    const int64_t tile_sz = kWave;
    const int64_t n_tiles = (n + tile_sz - 1) / tile_sz;
    const LaunchInfo info = *a.ws.info;
    const R dtr = (R)a.st.dt;
    const R *rec = (const R *)a.ws.stage.rec;
    const int64_t slots = a.ws.stage.slots;
    const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave, lane = lane_id();
    int cnt[N_COUNT_USED];
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) cnt[k] = 0;
    // one chunk of records per wave (XCD-contiguous ranges of chunks)
    for (int64_t it = wid;; it += nw) {
        const int64_t tile = xcd_tile(it, n_tiles);
        if (tile < 0) break;
        const uint32_t nrec = a.ws.stage.n_rec[tile];
        if (nrec == 0u) continue;
        uint32_t base0 = a.ws.tile_pre0[tile], base1 = a.ws.tile_pre1[tile];
        for (uint32_t r0 = 0; r0 < nrec; r0 += kWave) {    // one round: chunks hold 64 records
            const uint32_t r = r0 + (uint32_t)lane;
            const bool have = r < nrec;
            const int64_t sl = tile * tile_sz + r;
            uint32_t meta = 0, c0 = 0, c1 = 0;
            if (have) {
                meta = a.ws.stage.meta[sl];
                const uint32_t ne = meta & 7u;
#pragma unroll
                for (int k = 0; k < kMaxEvents; ++k)
                    if ((uint32_t)k < ne) {
                        const uint32_t d = (meta >> (3 + 2 * k)) & 3u;
                        c0 += d == 0u;
                        c1 += d == 1u;
                    }
            }
            // both counts in one scan: at most 4 x 256 per tile, so 16 bits each
            uint32_t tot;
            const uint32_t ex = wave_excl_scan(c0 | (c1 << 16), tot);
            if (have) {
                uint32_t g0 = base0 + (ex & 0xffffu), g1 = base1 + (ex >> 16);
                const R x0 = rec[0 * slots + sl], y0 = rec[1 * slots + sl], z0 = rec[2 * slots + sl];
                const R hx = rec[3 * slots + sl], hy = rec[4 * slots + sl], hz = rec[5 * slots + sl];
                const R wgt = rec[6 * slots + sl];
                const uint32_t ne = meta & 7u;
#pragma unroll
                for (int k = 0; k < kMaxEvents; ++k) {
                    if ((uint32_t)k >= ne) break;
                    const uint32_t d = (meta >> (3 + 2 * k)) & 3u;
                    if (d > 1u) continue;
                    const uint64_t nid = info.uid0 + (uint64_t)g0 + (uint64_t)g1;
                    const SpeciesDev &S = d == 0u ? a.pp : a.pr;
                    const int64_t j = d == 0u ? info.base0 + (int64_t)g0 : info.base1 + (int64_t)g1;
                    if (d == 0u) ++g0; else ++g1;
                    if (j >= S.cap) { cnt[C_LOST]++; continue; }
                    const R gg = rec[(7 + k) * slots + sl];
                    ((R *)S.x)[j] = x0 + dtr * hx;
                    ((R *)S.y)[j] = y0 + dtr * hy;
                    ((R *)S.z)[j] = z0 + dtr * hz;
                    ((R *)S.ux)[j] = gg * hx;
                    ((R *)S.uy)[j] = gg * hy;
                    ((R *)S.uz)[j] = gg * hz;
                    ((R *)S.w)[j] = wgt;
                    if (S.chi) ((R *)S.chi)[j] = rec[(11 + k) * slots + sl];
                    S.uid[j] = nid;
                    S.n_ev[j] = 0u;
                    S.tau[j] = initial_tau(a.st.seed, nid);
                }
            }
            base0 += tot & 0xffffu;
            base1 += tot >> 16;
        }
    }
    block_counts(a.tal, cnt, s_cnt);
}

// ------------------------------------------------------------------------
// Photon step: Breit-Wheeler pair creation (Sec. 3, Eq. 3) and straight-line
// push.  The physics pass marks a photon that decays with tau = -inf and
// leaves its position and momentum as they were; the append pass recomputes
// the decay of marked photons, writes the pair and sets tau = +inf (removed
// later by k_compact).
// ------------------------------------------------------------------------
//
// Blocks take chunks of blockDim.x photons (XCD-contiguous ranges of chunks);
// each wave of a block steps its own tile of 64 photons of the chunk and
// publishes that tile's pair count, so the loop has no block barrier.  The
// state of a wave's next tile is loaded before the current one is stepped,
// which hides the HBM latency behind the gather.
template <typename R, int FK, bool kCull>
__global__ void __launch_bounds__(256)
k_pair_create(PairArgs a) {
    __shared__ R s_lp[kMaxChiNodes];
    __shared__ float s_box[FK == FIELD_YEE ? kMaxWaves * kWBFloats : 1];
    __shared__ int64_t s_cnt[N_COUNT_USED];

    const int tid = threadIdx.x, lane = lane_id(), nw = blockDim.x / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);    // uniform over the wave
    const TablesDev &tb = a.tab;
    for (int i = tid; i < tb.p_n_chi; i += blockDim.x) s_lp[i] = (R)tb.pair_lnh[i];
    const int64_t n = *a.ph.count;
    const double t = a.st.d_step ? a.st.t + (double)(*a.st.d_step) * a.st.dt : a.st.t;
    const double dt = a.st.dt;
    const R dtr = (R)dt;
    const int64_t n_chunks = (n + blockDim.x - 1) / blockDim.x;
    const int64_t n_tiles = (n + kWave - 1) / kWave;
    const R es_inv = (R)a.c.es_inv, Ah = (R)a.c.A;
    const R lnchi0 = (R)tb.p_lnchi0, inv_d = (R)tb.p_inv_dlnchi, chi_min = (R)tb.p_chi_min;
    R *X = (R *)a.ph.x, *Y = (R *)a.ph.y, *Z = (R *)a.ph.z;
    const R *KX = (const R *)a.ph.ux, *KY = (const R *)a.ph.uy, *KZ = (const R *)a.ph.uz;
    int cnt[N_COUNT_USED];
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) cnt[k] = 0;
    __syncthreads();

    int64_t chunk = xcd_tile(0, n_chunks);
    double n_tau = HUGE_VAL;
    R n_x = R(0), n_y = R(0), n_z = R(0), n_kx = R(0), n_ky = R(0), n_kz = R(0);
    const uint32_t ul = (uint32_t)lane;
    if (chunk >= 0 && chunk * blockDim.x + tid < n) {
        const int64_t b = (chunk * nw + wid) * kWave;
        n_tau = wave_base(a.ph.tau, b)[ul];
        n_x = wave_base(X, b)[ul]; n_y = wave_base(Y, b)[ul]; n_z = wave_base(Z, b)[ul];
        n_kx = wave_base(KX, b)[ul]; n_ky = wave_base(KY, b)[ul]; n_kz = wave_base(KZ, b)[ul];
    }
    for (int64_t it = 0; chunk >= 0; ++it) {
        const int64_t tile = chunk * nw + wid;              // = i / 64
        const int64_t i = chunk * blockDim.x + tid;
        double en[kNEnergy];
#pragma unroll
        for (int k = 0; k < kNEnergy; ++k) en[k] = 0.0;
        bool event = false;
        double tau = n_tau;
        R x = n_x, y = n_y, z = n_z, kx = n_kx, ky = n_ky, kz = n_kz;
        const bool live = i < n && tau != HUGE_VAL;
        if (!live) x = y = z = kx = ky = kz = R(0);
        const int64_t next = xcd_tile(it + 1, n_chunks);
        auto prefetch = [&]() {
            n_tau = HUGE_VAL;
            if (next >= 0 && next * blockDim.x + tid < n) {
                const int64_t b = (next * nw + wid) * kWave;
                n_tau = wave_base(a.ph.tau, b)[ul];
                n_x = wave_base(X, b)[ul]; n_y = wave_base(Y, b)[ul]; n_z = wave_base(Z, b)[ul];
                n_kx = wave_base(KX, b)[ul]; n_ky = wave_base(KY, b)[ul]; n_kz = wave_base(KZ, b)[ul];
            }
        };
        // with a grid the loads go out after the gather's (whose wait would include them)
        if constexpr (FK != FIELD_YEE) prefetch();
        const int64_t tile0 = tile * kWave;                 // = i - lane
        // |k| = gamma_gamma, with one rounding order whatever the kernel variant
        const R kk = Math<R>::sqrt_(fma(kz, kz, fma(ky, ky, kx * kx)));
        R E[3], B[3], xn = R(0), yn = R(0), zn = R(0);
        if constexpr (FK == FIELD_YEE) {
            // a wave whose photons all have a pair rate of exactly zero whatever the
            // field skips the gather: chi_gamma <= |k| (|E| + |B|) / E_s, bounded over
            // the blocks of cells the wave spans with the largest |k| of the wave
            bool cull = false;
            if (kCull) {
                if (__ballot(live) == 0ull) {
                    cull = true;                                  // nothing to gather
                } else {
                    const double gc[3] = {((double)x - a.f.x0) * a.f.inv_dx, ((double)y - a.f.y0) * a.f.inv_dy,
                                          ((double)z - a.f.z0) * a.f.inv_dz};
                    const int64_t nc[3] = {a.f.nx, a.f.ny, a.f.nz};
                    int blo[3], nbk[3];
                    int64_t nblk = 1;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        // NaN positions land in cell 0: their pair rate is zero whatever the field
                        const double cl =
                            gc[d] > 0.0 ? (gc[d] < (double)(nc[d] - 1) ? gc[d] : (double)(nc[d] - 1)) : 0.0;
                        const int b = (int)((int64_t)cl / a.f.bb);
                        blo[d] = wave_min_i32(live ? b : INT_MAX);
                        const int bhi = -wave_min_i32(live ? -b : INT_MAX);
                        nbk[d] = bhi - blo[d] + 1;               // >= 1: some lane is live
                        nblk *= nbk[d];
                    }
                    if (nblk <= kWave) {
                        const double kd = live ? (double)kk : 0.0;
                        double kmax = kd, fmax_ = 0.0;
                        const int lane = lane_id();
                        if (lane < (int)nblk) {
                            const int bk = blo[2] + lane % nbk[2], bj = blo[1] + (lane / nbk[2]) % nbk[1],
                                      bi = blo[0] + lane / (nbk[2] * nbk[1]);
                            const float *bd = a.f.bound + 2 * (((int64_t)bi * a.f.nby + bj) * a.f.nbz + bk);
                            fmax_ = (double)bd[0] + (double)bd[1];
                        }
#pragma unroll
                        for (int o = kWave / 2; o > 0; o >>= 1) {
                            kmax = fmax(kmax, __shfl_xor(kmax, o, kWave));
                            fmax_ = fmax(fmax_, __shfl_xor(fmax_, o, kWave));
                        }
                        cull = kmax * fmax_ * a.c.es_inv * 1.01 < tb.p_chi_min;
                    }
                }
            }
            if (cull) {
#pragma unroll
                for (int d = 0; d < 3; ++d) { E[d] = R(0); B[d] = R(0); }
                if (live) cnt[C_NOGATHER]++;
                prefetch();
            } else {
                yee_gather_wave<R>(a.f, live, x, y, z, E, B, s_box + (tid / kWave) * kWBFloats, prefetch);
            }
        }
        if (live) {
            if constexpr (FK != FIELD_YEE) field_at<R, FK>(a.f, t, x, y, z, a.f.a0, a.f.Phi, a.f.inv_Phi, E, B);
            const R chig = chi_of<R>(es_inv, kk, kx, ky, kz, E, B);
            cnt[C_PHSTEP]++;
            R Wp = R(0);
            const R ik = Math<R>::rcp_(kk);
            if (kk > R(2) && chig >= chi_min) {
                bool above = false;
                const R l = lerp_rate<R>(s_lp, tb.p_n_chi, lnchi0, inv_d, Math<R>::log_(chig), above);
                Wp = Ah * Math<R>::exp_(l - R(8) / (R(3) * chig)) * ik;
                if (above) cnt[C_RANGE]++;
            }
            tau -= (double)Wp * dt;
            if (Wp > R(0) && tau <= 0.0) {
                event = true;
                cnt[C_PAIR]++;
                tau = -HUGE_VAL;
                en[E_PAIR] = (double)((const R *)a.ph.w)[i] * (double)kk;
            } else {
                xn = x + dtr * (kx * ik);
                yn = y + dtr * (ky * ik);
                zn = z + dtr * (kz * ik);
            }
        }
        // the next tile's loads are waited for before this tile's stores, not after
        // them (the memory counter retires in issue order)
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        if (live) {
            wave_base(a.ph.tau, tile0)[ul] = tau;
            if (!event) {
                wave_base(X, tile0)[ul] = xn; wave_base(Y, tile0)[ul] = yn; wave_base(Z, tile0)[ul] = zn;
            }
        }
        const uint32_t tot = (uint32_t)__popcll(__ballot(event));
        if (tile < n_tiles) {
            if (lane == 0) {
                a.ws.tile_cnt0[tile] = tot;
                a.ws.tile_cnt1[tile] = 0u;
            }
            wave_energy<kNEnergy>(a.tal, tile, en);
        }
        chunk = next;
    }
    block_counts(a.tal, cnt, s_cnt);
}

// Append pass of the photon step: e- and e+ of each marked photon (kSpline as
// for the lepton event pass).
template <typename R, int FK, bool kSpline>
__global__ void __launch_bounds__(256)
k_pair_append(PairArgs a) {
    __shared__ uint32_t s_wave[3 * kMaxWaves];
    __shared__ uint32_t s_list[256];
    __shared__ int64_t s_cnt[N_COUNT_USED];
    const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave, lane = lane_id();
    const TablesDev &tb = a.tab;
    const int64_t n = *a.ph.count;
    const int64_t tile_sz = a.tile_sz;                 // kWave: one wave per physics tile
    const int64_t n_tiles = (n + tile_sz - 1) / tile_sz;
    const int64_t n_chunks = (n_tiles + blockDim.x - 1) / blockDim.x;
    const LaunchInfo info = *a.ws.info;
    const double t = a.st.d_step ? a.st.t + (double)(*a.st.d_step) * a.st.dt : a.st.t;
    const R dtr = (R)a.st.dt;
    const R es_inv = (R)a.c.es_inv;
    const R lnchi0 = (R)tb.p_lnchi0, inv_d = (R)tb.p_inv_dlnchi;
    const R *qtab = pair_q_ptr<R>(tb), *qspl = kSpline ? pair_qs_ptr<R>(tb) : nullptr;
    int cnt[N_COUNT_USED];
#pragma unroll
    for (int k = 0; k < N_COUNT_USED; ++k) cnt[k] = 0;
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        // tiles are one wave (64 photons) in the physics pass: each wave takes its
        // own listed tiles and ranks their pairs with a ballot, with no block barrier
        const uint32_t m = list_tiles(a.ws.tile_cnt0, c, n_tiles, s_list, s_wave);
        for (uint32_t qi = (uint32_t)wid; qi < m; qi += (uint32_t)nw) {
            const int64_t tile = c * blockDim.x + s_list[qi];
            const int64_t i = tile * tile_sz + lane;
            const bool ev = i < n && a.ph.tau[i] == -HUGE_VAL;
            uint32_t tot;
            const uint32_t e = ballot_excl(ev, tot);
            if (ev) {
                const R x = ((const R *)a.ph.x)[i], y = ((const R *)a.ph.y)[i], z = ((const R *)a.ph.z)[i];
                const R kx = ((const R *)a.ph.ux)[i], ky = ((const R *)a.ph.uy)[i], kz = ((const R *)a.ph.uz)[i];
                const R wgt = ((const R *)a.ph.w)[i];
                R E[3], B[3];
                field_at<R, FK>(a.f, t, x, y, z, a.f.a0, a.f.Phi, a.f.inv_Phi, E, B);
                const R kk = Math<R>::sqrt_(fma(kz, kz, fma(ky, ky, kx * kx)));     // as in the physics pass
                const R chig = chi_of<R>(es_inv, kk, kx, ky, kz, E, B);
                const R khx = kx / kk, khy = ky / kk, khz = kz / kk;
                const U64x4 o = philox4x64_10(a.ph.uid[i], (uint64_t)a.ph.n_ev[i], (uint64_t)RNG_PAIR, 0ull,
                                              a.st.seed, 0ull);
                const R s = quantile<R>(qtab, qspl, (R)tb.p_ht26, (R)tb.p_hc26, tb.p_n_chi, tb.p_n_q, lnchi0,
                                        inv_d, tb.p_logit_max, tb.p_inv_dt, Math<R>::log_(chig), u01(o.a));
                const R eta = R(1) / (R(1) + Math<R>::exp_(-s));
                const R chim = eta * chig;
                const R chip = chig - chim;
                // default: energy split exactly along k; variant: momentum split exactly
                const bool pmom = (a.st.variants & VAR_PAIR_MOMENTUM) != 0;
                const R pm_m = (chim / chig) * kk, pm_p = (chip / chig) * kk;
                const R gmn = pmom ? Math<R>::sqrt_(R(1) + pm_m * pm_m) : R(1) + (kk - R(2)) * (chim / chig);
                const R gpl = pmom ? Math<R>::sqrt_(R(1) + pm_p * pm_p) : R(1) + (kk - R(2)) * (chip / chig);
                const uint32_t g = a.ws.tile_pre0[tile] + e;
                const uint64_t nid = info.uid0 + 2ull * (uint64_t)g;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const SpeciesDev &D = side == 0 ? a.el : a.po;
                    const int64_t j = (side == 0 ? info.base0 : info.base1) + (int64_t)g;
                    if (j >= D.cap) { cnt[C_LOST]++; continue; }
                    const R gmag = side == 0 ? gmn : gpl;
                    const R pm = pmom ? (side == 0 ? pm_m : pm_p) : Math<R>::sqrt_(gmag * gmag - R(1));
                    const R ux = pm * khx, uy = pm * khy, uz = pm * khz;
                    const uint64_t id = nid + (uint64_t)side;
                    ((R *)D.x)[j] = x + dtr * (ux / gmag);
                    ((R *)D.y)[j] = y + dtr * (uy / gmag);
                    ((R *)D.z)[j] = z + dtr * (uz / gmag);
                    ((R *)D.ux)[j] = ux;
                    ((R *)D.uy)[j] = uy;
                    ((R *)D.uz)[j] = uz;
                    ((R *)D.w)[j] = wgt;
                    if (D.chi) ((R *)D.chi)[j] = side == 0 ? chim : chip;
                    D.uid[j] = id;
                    D.n_ev[j] = 0u;
                    D.tau[j] = initial_tau(a.st.seed, id);
                }
                a.ph.tau[i] = HUGE_VAL;
            }
        }
        __syncthreads();       // s_list is rewritten for the next chunk only after every wave is done
    }
    block_counts(a.tal, cnt, s_cnt);
}

// ------------------------------------------------------------------------
// Stable in-place compaction of the photons that are still alive.  Every
// thread holds its whole particle in registers before the tile publishes its
// count, so a later tile writing over this tile's slots cannot clobber data
// that has not been read yet.
// ------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256)
k_compact(CompactArgs a) {
    constexpr int kItems = 4;                          // tiles of kItems x blockDim.x photons
    __shared__ uint64_t s_ticket;
    __shared__ uint32_t s_wc[kItems * kMaxWaves];      // alive photons per (item row, wave)
    __shared__ uint32_t s_pref;
    const int tid = threadIdx.x, lane = lane_id(), nw = blockDim.x / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);    // uniform over the wave
    const int64_t n = *a.s.count;
    const int64_t tile_sz = (int64_t)blockDim.x * kItems;
    const int64_t n_tiles = (n + tile_sz - 1) / tile_sz;
    R *X = (R *)a.s.x, *Y = (R *)a.s.y, *Z = (R *)a.s.z;
    R *UX = (R *)a.s.ux, *UY = (R *)a.s.uy, *UZ = (R *)a.s.uz, *Wt = (R *)a.s.w, *CH = (R *)a.s.chi;
    __syncthreads();
    for (;;) {
        if (tid == 0) s_ticket = atomicAdd((unsigned long long *)a.ws.ticket, 1ull);
        __syncthreads();
        const uint64_t tk = s_ticket;
        const uint32_t epoch = (uint32_t)(tk >> 32);
        const int64_t tile = (int64_t)(tk & 0xffffffffull);
        if (tile >= n_tiles) {
            if (tid == 0 && tile == n_tiles + (int64_t)gridDim.x - 1) {
                if (n_tiles > 0) {
                    uint32_t t0, t1;
                    lb_wait_inclusive(a.ws.lb, n_tiles - 1, epoch, t0, t1);
                    *a.s.count = (int64_t)t0;
                }
                atomicAdd((unsigned long long *)a.ws.ticket,
                          (1ull << 32) - (unsigned long long)(n_tiles + (int64_t)gridDim.x));
            }
            break;
        }
        // photon u * blockDim.x + tid of the tile: coalesced rows, kept in index order
        const int64_t base = tile * tile_sz;
        bool alive[kItems];
        R x[kItems], y[kItems], z[kItems], ux[kItems], uy[kItems], uz[kItems], w[kItems], ch[kItems];
        double tau[kItems];
        uint64_t uid[kItems];
        uint32_t nev[kItems];
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + tid;
            alive[u] = false;
            x[u] = y[u] = z[u] = ux[u] = uy[u] = uz[u] = w[u] = ch[u] = R(0);
            tau[u] = 0.0; uid[u] = 0; nev[u] = 0;
            if (i < n) {
                tau[u] = a.s.tau[i];
                alive[u] = tau[u] != HUGE_VAL;
                if (alive[u]) {
                    x[u] = X[i]; y[u] = Y[i]; z[u] = Z[i]; ux[u] = UX[i]; uy[u] = UY[i]; uz[u] = UZ[i]; w[u] = Wt[i];
                    if (CH) ch[u] = CH[i];
                    uid[u] = a.s.uid[i];
                    nev[u] = a.s.n_ev[i];
                }
            }
        }
        // all loads of this tile complete before its count becomes visible
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        uint64_t m[kItems];
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            m[u] = __ballot(alive[u]);
            if (lane == 0) s_wc[u * kMaxWaves + wid] = (uint32_t)__popcll(m[u]);
        }
        __syncthreads();
        // rank of photon (u, tid): alive photons in earlier rows, then in earlier waves of row u
        uint32_t before[kItems], tot = 0;
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            uint32_t r = tot;
            for (int v = 0; v < nw; ++v) {
                const uint32_t c = s_wc[u * kMaxWaves + v];
                if (v < wid) r += c;
                tot += c;
            }
            before[u] = r + __builtin_amdgcn_mbcnt_hi((uint32_t)(m[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[u], 0u));
        }
        if (tid < kWave) {
            uint32_t p0, p1;
            lookback2(a.ws.lb, tile, epoch, tot, 0u, p0, p1);
            if (tid == 0) s_pref = p0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + tid;
            if (alive[u]) {
                const int64_t j = (int64_t)(s_pref + before[u]);
                if (j != i) {
                    X[j] = x[u]; Y[j] = y[u]; Z[j] = z[u]; UX[j] = ux[u]; UY[j] = uy[u]; UZ[j] = uz[u]; Wt[j] = w[u];
                    if (CH) CH[j] = ch[u];
                    a.s.uid[j] = uid[u];
                    a.s.n_ev[j] = nev[u];
                    a.s.tau[j] = tau[u];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// small kernels
// ------------------------------------------------------------------------
__global__ void k_init_tau(const uint64_t *uid, double *tau, const int64_t *count, uint64_t seed) {
    const int64_t n = *count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        tau[i] = initial_tau(seed, uid[i]);
}

__global__ void k_yee_fill(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                           const double *tperp, const double *tpar) {
    const int64_t plane = ny * nz, ncell = nx * plane, total = 6 * ncell;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx / ncell, r = idx - c * ncell;
        const int64_t i = r / plane, jk = r - i * plane;
        grid[idx] = (float)((a0 * tperp[c * plane + jk]) * tpar[c * nx + i]);
    }
}

// Per-block field bounds: thread (block, E or B) takes the largest |component|
// of each of its three components over the block's nodes and two more on
// every side, and stores sqrt of the sum of their squares (rounded up).
__global__ void __launch_bounds__(256)
k_field_bound(const float *grid, int64_t nx, int64_t ny, int64_t nz, int64_t bb, int64_t nbx, int64_t nby,
              int64_t nbz, float *bound) {
    const int64_t nb = nbx * nby * nbz, ncell = nx * ny * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 2 * nb; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t >> 1;
        const int fb = (int)(t & 1);
        const int64_t bk = b % nbz, bj = (b / nbz) % nby, bi = b / (nbz * nby);
        const int64_t i0 = bi * bb - 2 < 0 ? 0 : bi * bb - 2, i1 = bi * bb + bb + 2 > nx ? nx : bi * bb + bb + 2;
        const int64_t j0 = bj * bb - 2 < 0 ? 0 : bj * bb - 2, j1 = bj * bb + bb + 2 > ny ? ny : bj * bb + bb + 2;
        const int64_t k0 = bk * bb - 2 < 0 ? 0 : bk * bb - 2, k1 = bk * bb + bb + 2 > nz ? nz : bk * bb + bb + 2;
        double s2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const float *g = grid + (int64_t)(3 * fb + c) * ncell;
            float m = 0.0f;
            for (int64_t i = i0; i < i1; ++i)
                for (int64_t j = j0; j < j1; ++j) {
                    const float *r = g + (i * ny + j) * nz;
                    for (int64_t k = k0; k < k1; ++k) m = fmaxf(m, fabsf(r[k]));
                }
            s2 += (double)m * (double)m;
        }
        // NaN anywhere in the region leaves the bound infinite (no cull)
        bound[t] = isfinite(s2) ? (float)(sqrt(s2) * (1.0 + 0x1p-20)) : HUGE_VALF;
    }
}

hipError_t launch_field_bound(const float *grid, int64_t nx, int64_t ny, int64_t nz, int64_t block, float *bound,
                              hipStream_t s) {
    const int64_t nbx = (nx + block - 1) / block, nby = (ny + block - 1) / block, nbz = (nz + block - 1) / block;
    const int64_t n = 2 * nbx * nby * nbz;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535));
    hipLaunchKernelGGL(k_field_bound, dim3(g), dim3(256), 0, s, grid, nx, ny, nz, block, nbx, nby, nbz, bound);
    return hipGetLastError();
}

__global__ void k_step_advance(int64_t *d_step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_step += 1;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <typename R>
hipError_t launch_stream(const PushArgs &a, int fk, dim3 grid, dim3 block, hipStream_t s) {
    switch (fk) {
    case FIELD_UNIFORM: hipLaunchKernelGGL((k_lepton_stream<R, FIELD_UNIFORM>), grid, block, 0, s, a); break;
    case FIELD_PLANE: hipLaunchKernelGGL((k_lepton_stream<R, FIELD_PLANE>), grid, block, 0, s, a); break;
    case FIELD_YEE: hipLaunchKernelGGL((k_lepton_stream<R, FIELD_YEE>), grid, block, 0, s, a); break;
    default:
        if (a.f.lds_bunches)
            hipLaunchKernelGGL((k_lepton_stream<R, FIELD_BUNCHED>), grid, block,
                               (size_t)lds_bunch_bytes(a.f.n_bunches), s, a);
        else
            hipLaunchKernelGGL((k_lepton_stream<R, FIELD_BUNCHED_GLOBAL>), grid, block, 0, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_lepton_stream(const PushArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s) {
    return prec == 0 ? launch_stream<double>(a, fk, grid, block, s) : launch_stream<float>(a, fk, grid, block, s);
}

hipError_t launch_lepton_events(const PushArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s) {
    const bool spl = a.tab.emit_qs != nullptr;
    if (prec == 0) {
        if (spl) hipLaunchKernelGGL((k_lepton_events<double, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_lepton_events<double, false>), grid, block, 0, s, a);
    } else {
        if (spl) hipLaunchKernelGGL((k_lepton_events<float, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_lepton_events<float, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_scan_tiles(const ScanArgs &a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_tiles, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_push_append(const PushArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s) {
    if (prec == 0) hipLaunchKernelGGL((k_push_append<double>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_push_append<float>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pair(const PairArgs &a, int fk, dim3 grid, dim3 block, hipStream_t s) {
    switch (fk) {
    case FIELD_UNIFORM: hipLaunchKernelGGL((k_pair_create<R, FIELD_UNIFORM, false>), grid, block, 0, s, a); break;
    case FIELD_PLANE: hipLaunchKernelGGL((k_pair_create<R, FIELD_PLANE, false>), grid, block, 0, s, a); break;
    default:
        // the field-bound cull is a separate instantiation, so that the plain gather keeps its registers
        if (a.f.bound) hipLaunchKernelGGL((k_pair_create<R, FIELD_YEE, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_pair_create<R, FIELD_YEE, false>), grid, block, 0, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_pair_create(const PairArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s) {
    return prec == 0 ? launch_pair<double>(a, fk, grid, block, s) : launch_pair<float>(a, fk, grid, block, s);
}

template <typename R, bool kSpline>
hipError_t launch_pair_app(const PairArgs &a, int fk, dim3 grid, dim3 block, hipStream_t s) {
    switch (fk) {
    case FIELD_UNIFORM: hipLaunchKernelGGL((k_pair_append<R, FIELD_UNIFORM, kSpline>), grid, block, 0, s, a); break;
    case FIELD_PLANE: hipLaunchKernelGGL((k_pair_append<R, FIELD_PLANE, kSpline>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_pair_append<R, FIELD_YEE, kSpline>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_pair_append(const PairArgs &a, int prec, int fk, dim3 grid, dim3 block, hipStream_t s) {
    if (a.tab.pair_qs != nullptr)
        return prec == 0 ? launch_pair_app<double, true>(a, fk, grid, block, s)
                         : launch_pair_app<float, true>(a, fk, grid, block, s);
    return prec == 0 ? launch_pair_app<double, false>(a, fk, grid, block, s)
                     : launch_pair_app<float, false>(a, fk, grid, block, s);
}

hipError_t launch_compact(const CompactArgs &a, int prec, dim3 grid, dim3 block, hipStream_t s) {
    if (prec == 0) hipLaunchKernelGGL((k_compact<double>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_compact<float>), grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_tau(const uint64_t *uid, double *tau, const int64_t *count, uint64_t seed,
                           int n_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_init_tau, dim3(n_blocks), dim3(256), 0, s, uid, tau, count, seed);
    return hipGetLastError();
}

hipError_t launch_yee_fill(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                           const double *tperp, const double *tpar, int n_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_yee_fill, dim3(n_blocks), dim3(256), 0, s, grid, nx, ny, nz, a0, tperp, tpar);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Log-binned spectrum: per-block LDS histograms of counts and of integer
// (fixed-point) weights, added to the global bins once per block.  Integer
// additions commute, so the result does not depend on the schedule.
// ------------------------------------------------------------------------
constexpr int kMaxSpecBins = 1024 + 2;

template <typename R>
__global__ void __launch_bounds__(256)
k_spectrum(SpectrumArgs a) {
    __shared__ unsigned long long s_c[kMaxSpecBins], s_w[kMaxSpecBins];
    const int nb = a.n_bins + 2;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) { s_c[b] = 0ull; s_w[b] = 0ull; }
    __syncthreads();
    const int64_t n = *a.s.count < a.s.cap ? *a.s.count : a.s.cap;
    const R *UX = (const R *)a.s.ux, *UY = (const R *)a.s.uy, *UZ = (const R *)a.s.uz, *W = (const R *)a.s.w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double tau = a.s.tau[i];
        if (a.photons && (tau == HUGE_VAL || tau == -HUGE_VAL)) continue;
        const double ux = (double)UX[i], uy = (double)UY[i], uz = (double)UZ[i];
        const double u2 = ux * ux + uy * uy + uz * uz;
        const double e = a.photons ? sqrt(u2) : sqrt(1.0 + u2);
        int b = 0;
        if (e >= a.e_max) {
            b = a.n_bins + 1;
        } else if (e >= a.e_min) {
            const double f = floor((log(e) - a.ln_emin) * a.inv_dln);
            b = 1 + (f < 0.0 ? 0 : (f >= (double)a.n_bins ? a.n_bins - 1 : (int)f));
        }
        const long long wf = llrint((double)W[i] * a.wscale);
        atomicAdd(&s_c[b], 1ull);
        atomicAdd(&s_w[b], (unsigned long long)wf);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        if (s_c[b]) {
            atomicAdd(a.count + b, s_c[b]);
            atomicAdd(a.wsum + b, s_w[b]);
        }
    }
}

hipError_t launch_spectrum(const SpectrumArgs &a, int prec, int n_blocks, hipStream_t s) {
    if (prec == 0) hipLaunchKernelGGL((k_spectrum<double>), dim3(n_blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_spectrum<float>), dim3(n_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_step_advance(int64_t *d_step, hipStream_t s) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, d_step);
    return hipGetLastError();
}

}  // namespace qed
