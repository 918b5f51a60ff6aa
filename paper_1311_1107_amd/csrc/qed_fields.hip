// qed_fields.hip -- Yee field solver and charge-conserving current deposition,
// the two pieces that couple the QED step to a particle-in-cell loop.
//
// Field solver: Yee's staggered finite differences in normalised units
// (c = 1), dB/dt = -curl E, dE/dt = curl B - J, periodic in every direction,
// FP32 like the grid [Ex Ey Ez Bx By Bz][nx][ny][nz] (z fastest) that the
// field gather reads.  One advance is B by dt/2, E by dt, B by dt/2, so that
// E and B sit at whole steps for the push.  Each update is one thread per
// cell with the same fmaf order as the oracle, so results are bit-identical.
//
// Deposition: Esirkepov's charge-conserving scheme with quadratic (TSC)
// shapes (Comput. Phys. Commun. 135, 144 (2001)).  Per particle the change of
// its node charges over the step, on a 5 x 5 x 5 window around the starting
// node, is split as W_x + W_y + W_z with
//   W_x = D_x (S_y S_z + D_y S_z / 2 + S_y D_z / 2 + D_y D_z / 3)
// (S the starting TSC weights, D the change), and J_x at the faces of the
// window is the running sum of -Q dx/dt W_x along x.  Shapes and sums are
// FP64; each face value is added to the FP32 current grid with a hardware
// float atomic, so the order of the additions (and the last bits of J) vary
// from run to run.  A particle whose nearest node moves by more than one
// cell in some direction (a step above the Courant limit) is skipped and
// counted.
#include <algorithm>
#include <climits>

#include "qed_fields.h"

namespace qed {

__device__ __forceinline__ int64_t count_clamped(const int64_t *count, int64_t cap) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

__device__ __forceinline__ int64_t wrapi(int64_t i, int64_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}

__global__ void __launch_bounds__(256)
k_yee_b_half(float *g, int64_t nx, int64_t ny, int64_t nz, float cx, float cy, float cz) {
    const int64_t N = nx * ny * nz;
    const float *Ex = g, *Ey = g + N, *Ez = g + 2 * N;
    float *Bx = g + 3 * N, *By = g + 4 * N, *Bz = g + 5 * N;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = c % nz, j = (c / nz) % ny, i = c / (nz * ny);
        const int64_t ip = c + ((i + 1 < nx) ? ny * nz : -(nx - 1) * ny * nz);
        const int64_t jp = c + ((j + 1 < ny) ? nz : -(ny - 1) * nz);
        const int64_t kp = c + ((k + 1 < nz) ? 1 : -(nz - 1));
        const float ex = Ex[c], ey = Ey[c], ez = Ez[c];
        Bx[c] = fmaf(cz, Ey[kp] - ey, fmaf(-cy, Ez[jp] - ez, Bx[c]));
        By[c] = fmaf(cx, Ez[ip] - ez, fmaf(-cz, Ex[kp] - ex, By[c]));
        Bz[c] = fmaf(cy, Ex[jp] - ex, fmaf(-cx, Ey[ip] - ey, Bz[c]));
    }
}

__global__ void __launch_bounds__(256)
k_yee_e_full(float *g, const float *J, int64_t nx, int64_t ny, int64_t nz, float cx, float cy, float cz, float dt) {
    const int64_t N = nx * ny * nz;
    float *Ex = g, *Ey = g + N, *Ez = g + 2 * N;
    const float *Bx = g + 3 * N, *By = g + 4 * N, *Bz = g + 5 * N;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = c % nz, j = (c / nz) % ny, i = c / (nz * ny);
        const int64_t im = c - ((i > 0) ? ny * nz : -(nx - 1) * ny * nz);
        const int64_t jm = c - ((j > 0) ? nz : -(ny - 1) * nz);
        const int64_t km = c - ((k > 0) ? 1 : -(nz - 1));
        const float jx = J ? J[c] : 0.0f, jy = J ? J[N + c] : 0.0f, jz = J ? J[2 * N + c] : 0.0f;
        const float bx = Bx[c], by = By[c], bz = Bz[c];
        Ex[c] = fmaf(cy, bz - Bz[jm], fmaf(-cz, by - By[km], fmaf(-dt, jx, Ex[c])));
        Ey[c] = fmaf(cz, bx - Bx[km], fmaf(-cx, bz - Bz[im], fmaf(-dt, jy, Ey[c])));
        Ez[c] = fmaf(cx, by - By[im], fmaf(-cy, bx - Bx[jm], fmaf(-dt, jz, Ez[c])));
    }
}

hipError_t launch_yee_advance(float *grid, const float *J, const GridGeom &g, double dt, int n_cu, hipStream_t s) {
    const int64_t N = g.nx * g.ny * g.nz;
    const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (int64_t)n_cu * 32));
    const float hx = (float)(0.5 * dt / g.dx), hy = (float)(0.5 * dt / g.dy), hz = (float)(0.5 * dt / g.dz);
    const float fx = (float)(dt / g.dx), fy = (float)(dt / g.dy), fz = (float)(dt / g.dz);
    hipLaunchKernelGGL(k_yee_b_half, dim3(gb), dim3(256), 0, s, grid, g.nx, g.ny, g.nz, hx, hy, hz);
    hipLaunchKernelGGL(k_yee_e_full, dim3(gb), dim3(256), 0, s, grid, J, g.nx, g.ny, g.nz, fx, fy, fz, (float)dt);
    hipLaunchKernelGGL(k_yee_b_half, dim3(gb), dim3(256), 0, s, grid, g.nx, g.ny, g.nz, hx, hy, hz);
    return hipGetLastError();
}

// TSC weights of grid coordinate u around its nearest node (returned)
__device__ __forceinline__ int64_t tsc_node(double u, double s[3]) {
    const double fn = floor(u + 0.5);
    const double d = u - fn;
    s[0] = 0.5 * (0.5 - d) * (0.5 - d);
    s[1] = 0.75 - d * d;
    s[2] = 0.5 * (0.5 + d) * (0.5 + d);
    return (int64_t)fn;
}

__device__ __forceinline__ bool coord_ok(double u) { return u > -1.0e15 && u < 1.0e15; }

__device__ __forceinline__ int wave_min_int(int v) {
    // row minima through DPP (quad permutations, row rotations), then the four
    // rows; the wave must be fully active
    auto mn = [](int a, int b) { return a < b ? a : b; };
    v = mn(v, __builtin_amdgcn_update_dpp(v, v, 0xb1, 0xf, 0xf, false));    // quad_perm 1,0,3,2
    v = mn(v, __builtin_amdgcn_update_dpp(v, v, 0x4e, 0xf, 0xf, false));    // quad_perm 2,3,0,1
    v = mn(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false));   // row_ror 4
    v = mn(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false));   // row_ror 8
    return mn(mn(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
              mn(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Per-particle stencil of the deposition: window start (node n0 - 2 per axis),
// starting TSC weights S0 and their change D on the 5-node window.
struct DepStencil {
    double S0[3][5], D[3][5];
    int64_t base[3];
    int lo[3], hi[3];                // first window node of the support, last face with current
    double Q;
};

template <typename R>
__device__ __forceinline__ bool deposit_stencil(const DepositArgs &a, int64_t p, int64_t first, DepStencil &st) {
    const R *X = (const R *)a.s.x, *Y = (const R *)a.s.y, *Z = (const R *)a.s.z;
    const R *XO = (const R *)a.xo, *YO = (const R *)a.yo, *ZO = (const R *)a.zo;
    const double xn[3] = {(double)X[p], (double)Y[p], (double)Z[p]};
    double xb[3];
    if (XO) {
        xb[0] = (double)XO[p - first]; xb[1] = (double)YO[p - first]; xb[2] = (double)ZO[p - first];
    } else {
        const R *UX = (const R *)a.s.ux, *UY = (const R *)a.s.uy, *UZ = (const R *)a.s.uz;
        const double u0 = (double)UX[p], u1 = (double)UY[p], u2 = (double)UZ[p];
        const double ig = 1.0 / sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2);
        xb[0] = xn[0] - a.dt * (u0 * ig);
        xb[1] = xn[1] - a.dt * (u1 * ig);
        xb[2] = xn[2] - a.dt * (u2 * ig);
    }
    const double org[3] = {a.g.x0, a.g.y0, a.g.z0}, inv[3] = {a.g.inv_dx, a.g.inv_dy, a.g.inv_dz};
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g0 = (xb[c] - org[c]) * inv[c], g1 = (xn[c] - org[c]) * inv[c];
        double s0[3], s1[3];
        ok = ok && coord_ok(g0) && coord_ok(g1);
        const int64_t n0 = tsc_node(ok ? g0 : 0.0, s0), n1 = tsc_node(ok ? g1 : 0.0, s1);
        const int64_t sh = n1 - n0;
        ok = ok && sh >= -1 && sh <= 1;
        st.base[c] = n0 - 2;
        // weights live on window nodes [lo, lo + 3]: lo = 1 + min(sh, 0); current flows
        // through faces lo .. hi, hi = 2 + max(sh, 0) (face q lies between nodes q and q + 1)
        st.lo[c] = sh < 0 ? 0 : 1;
        st.hi[c] = sh > 0 ? 3 : 2;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int i0 = q - 1, i1 = q - 1 - (int)sh;
            const double v0 = (i0 >= 0 && i0 < 3) ? s0[i0] : 0.0;
            const double v1 = (i1 >= 0 && i1 < 3) ? s1[i1] : 0.0;
            st.S0[c][q] = v0;
            st.D[c][q] = v1 - v0;
        }
    }
    st.Q = a.q_scale * (double)((const R *)a.s.w)[p];
    return ok;
}

// The face currents of one particle, handed to add(comp, i, j, k, value) with
// window-relative node offsets (0..4); J_c is the running sum of
// -Q d_c/dt W_c along c.  Only the particle's support is visited: along each
// axis the start and end weights are nonzero on the 4 window nodes from
// lo = 1 + min(shift, 0) on, and the running sum along c vanishes before the
// first and from the last of them on (the changes sum to zero; the rounding
// residue of that sum is dropped), so 3 x 4 x 4 x 3 static slots cover it.
template <typename Add>
__device__ __forceinline__ void deposit_faces(const DepStencil &st, const double dd[3], double dt, Add add) {
    double S[3][4], Dl[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool s1 = st.lo[d] != 0;       // support starts at window node 1
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            S[d][m] = s1 ? st.S0[d][m + 1] : st.S0[d][m];
            Dl[d][m] = s1 ? st.D[d][m + 1] : st.D[d][m];
        }
    }
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
        const double f = -st.Q * dd[comp] / dt;
        const int nf = st.hi[comp] - st.lo[comp] + 1;      // faces carrying current: 2 or 3
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double t = S[a1][b] * S[a2][c] + 0.5 * Dl[a1][b] * S[a2][c] + 0.5 * S[a1][b] * Dl[a2][c]
                                 + Dl[a1][b] * Dl[a2][c] / 3.0;
                double acc = 0.0;
                int off[3];
                off[a1] = st.lo[a1] + b;
                off[a2] = st.lo[a2] + c;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    acc += f * Dl[comp][q] * t;
                    if (q >= nf || acc == 0.0) continue;
                    off[comp] = st.lo[comp] + q;
                    add(comp, off[0], off[1], off[2], acc);
                }
            }
    }
}

// Waves whose 64 particles start within a box of kDepBox nodes per axis
// (window included; particles in cell order) sum their faces in LDS first
// and add the box to the grid once; other waves add each face directly.
constexpr int kDepBox = 8;
constexpr int kDepBoxN = kDepBox * kDepBox * kDepBox;

template <typename R>
__global__ void __launch_bounds__(256)
k_deposit_current(DepositArgs a) {
    __shared__ float s_box[kMaxWaves][3 * kDepBoxN];
    const int64_t n = count_clamped(a.s.count, a.s.cap);
    const int64_t first0 = a.d_first ? *a.d_first : 0;
    const int64_t first = first0 > 0 ? first0 : 0;
    const int64_t N = a.g.nx * a.g.ny * a.g.nz;
    const int64_t nn[3] = {a.g.nx, a.g.ny, a.g.nz};
    const double dd[3] = {a.g.dx, a.g.dy, a.g.dz};
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    float *box = s_box[wv];
    uint32_t skipped = 0;
    const int64_t wstride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w0 = first + ((int64_t)blockIdx.x * (blockDim.x / kWave) + wv) * kWave; w0 < n; w0 += wstride) {
        const int64_t p = w0 + lane;
        const bool active = p < n && a.s.tau[p] != HUGE_VAL;
        DepStencil st;
        bool ok = false;
        if (active) {
            ok = deposit_stencil<R>(a, p, first, st);
            if (!ok) ++skipped;
        }
        const bool boxable = ok && st.base[0] > -(1 << 29) && st.base[0] < (1 << 29) && st.base[1] > -(1 << 29) &&
                             st.base[1] < (1 << 29) && st.base[2] > -(1 << 29) && st.base[2] < (1 << 29);
        int o[3];
        bool fits = __ballot(boxable) != 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[d] = wave_min_int(boxable ? (int)st.base[d] : INT_MAX);
            const int hi = -wave_min_int(boxable ? -(int)st.base[d] : INT_MAX);
            fits = fits && hi - o[d] + 5 <= kDepBox;
        }
        if (fits) {
            for (int e = lane; e < 3 * kDepBoxN; e += kWave) box[e] = 0.0f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (ok) {
            if (fits && boxable) {
                const int l0 = (int)st.base[0] - o[0], l1 = (int)st.base[1] - o[1], l2 = (int)st.base[2] - o[2];
                deposit_faces(st, dd, a.dt, [&](int comp, int i, int j, int k, double v) {
                    atomicAdd(box + comp * kDepBoxN + ((l0 + i) * kDepBox + (l1 + j)) * kDepBox + (l2 + k), (float)v);
                });
            } else {
                deposit_faces(st, dd, a.dt, [&](int comp, int i, int j, int k, double v) {
                    const int64_t ii = wrapi(st.base[0] + i, nn[0]), jj = wrapi(st.base[1] + j, nn[1]),
                                  kk = wrapi(st.base[2] + k, nn[2]);
                    unsafeAtomicAdd(a.out + comp * N + (ii * a.g.ny + jj) * a.g.nz + kk, (float)v);
                });
            }
        }
        if (fits) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int e = lane; e < 3 * kDepBoxN; e += kWave) {
                const float v = box[e];
                if (v == 0.0f) continue;
                const int comp = e / kDepBoxN, r = e % kDepBoxN;
                const int i = r / (kDepBox * kDepBox), j = (r / kDepBox) % kDepBox, k = r % kDepBox;
                const int64_t ii = wrapi((int64_t)o[0] + i, nn[0]), jj = wrapi((int64_t)o[1] + j, nn[1]),
                              kk = wrapi((int64_t)o[2] + k, nn[2]);
                unsafeAtomicAdd(a.out + comp * N + (ii * a.g.ny + jj) * a.g.nz + kk, v);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (a.skipped) {
        skipped = wave_sum_u32(skipped);
        if (lane == 0 && skipped) atomicAdd(a.skipped, (unsigned long long)skipped);
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_deposit_charge(DepositArgs a) {
    const int64_t n = count_clamped(a.s.count, a.s.cap);
    const R *X = (const R *)a.s.x, *Y = (const R *)a.s.y, *Z = (const R *)a.s.z, *Wt = (const R *)a.s.w;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if (a.s.tau[p] == HUGE_VAL) continue;
        const double g[3] = {((double)X[p] - a.g.x0) * a.g.inv_dx, ((double)Y[p] - a.g.y0) * a.g.inv_dy,
                             ((double)Z[p] - a.g.z0) * a.g.inv_dz};
        if (!coord_ok(g[0]) || !coord_ok(g[1]) || !coord_ok(g[2])) continue;
        double S[3][3];
        int64_t nd[3];
        for (int c = 0; c < 3; ++c) nd[c] = tsc_node(g[c], S[c]);
        const double Q = a.q_scale * (double)Wt[p];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) {
                    const int64_t ii = wrapi(nd[0] - 1 + i, a.g.nx), jj = wrapi(nd[1] - 1 + j, a.g.ny),
                                  kk = wrapi(nd[2] - 1 + k, a.g.nz);
                    unsafeAtomicAdd(a.out + (ii * a.g.ny + jj) * a.g.nz + kk, (float)(Q * S[0][i] * S[1][j] * S[2][k]));
                }
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_save_positions(SpeciesDev sp, R *xo, R *yo, R *zo) {
    const int64_t n = count_clamped(sp.count, sp.cap);
    const R *X = (const R *)sp.x, *Y = (const R *)sp.y, *Z = (const R *)sp.z;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        xo[p] = X[p];
        yo[p] = Y[p];
        zo[p] = Z[p];
    }
}

static unsigned particle_grid(int64_t cap, int n_cu) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + 255) / 256, (int64_t)n_cu * 16));
}

hipError_t launch_deposit_current(const DepositArgs &a, int prec, int n_cu, hipStream_t s) {
    const unsigned gb = particle_grid(a.s.cap, n_cu);
    if (prec == 0) hipLaunchKernelGGL((k_deposit_current<double>), dim3(gb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_deposit_current<float>), dim3(gb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_deposit_charge(const DepositArgs &a, int prec, int n_cu, hipStream_t s) {
    const unsigned gb = particle_grid(a.s.cap, n_cu);
    if (prec == 0) hipLaunchKernelGGL((k_deposit_charge<double>), dim3(gb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_deposit_charge<float>), dim3(gb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_save_positions(const SpeciesDev &sp, void *xo, void *yo, void *zo, int prec, int n_cu,
                                 hipStream_t s) {
    const unsigned gb = particle_grid(sp.cap, n_cu);
    if (prec == 0)
        hipLaunchKernelGGL((k_save_positions<double>), dim3(gb), dim3(256), 0, s, sp, (double *)xo, (double *)yo,
                           (double *)zo);
    else
        hipLaunchKernelGGL((k_save_positions<float>), dim3(gb), dim3(256), 0, s, sp, (float *)xo, (float *)yo,
                           (float *)zo);
    return hipGetLastError();
}

}  // namespace qed
