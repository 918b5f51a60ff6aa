// qed_device.h -- device building blocks of the QED step for gfx950 (CDNA4,
// wave64): counter-based random numbers, table lookups, field evaluation,
// quantum parameters, and the wave-ballot / decoupled look-back prefix sums
// used to append new particles in their parents' order.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace qed {

constexpr int kWave = 64;
constexpr int kMaxEvents = 4;     // emissions per particle and step
constexpr int kMaxChiNodes = 256;
constexpr int kMaxWaves = 4;      // 256 threads per block

enum { RNG_EMIT = 1, RNG_PAIR = 2, RNG_INIT = 3 };
// FIELD_BUNCHED_GLOBAL: the batched form with its bunch table read from global
// memory (a table too large for LDS); kernels only, never passed by the API
enum { FIELD_UNIFORM = 0, FIELD_PLANE = 1, FIELD_YEE = 2, FIELD_BUNCHED = 3, FIELD_BUNCHED_GLOBAL = 4 };
enum { RAD_NONE = 0, RAD_SOKOLOV = 1, RAD_MC = 2, RAD_HYBRID = 3 };

// count tallies (integer, accumulated per block across tiles)
enum { C_EMIT = 0, C_PUSH, C_REC, C_DROP, C_SUB, C_CAP, C_RANGE, C_SOKOLOV, C_MC,
       C_PAIR, C_PHSTEP, C_NAN, C_LOST, C_NOGATHER, N_COUNT_USED };
// energy tallies (FP64, per tile slot)
enum { E_WORK = 0, E_RAD, E_PUSH, E_REC, E_DROP, E_SUB, E_PAIR, N_ENERGY_USED };

constexpr double kPi = 3.141592653589793238462643383279502884;

// ------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplications; the key advances by the Weyl constants.
// ------------------------------------------------------------------------
struct U64x4 { uint64_t a, b, c, d; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return U64x4{c0, c1, c2, c3};
}

// uniform in ]0,1]: the paper's xi, xi', xi'' (Sec. 3)
__device__ __forceinline__ double u01(uint64_t bits) {
    return (double)((bits >> 11) + 1ull) * 0x1.0p-53;
}

// tau^f = -log xi for a newly created particle
__device__ __forceinline__ double initial_tau(uint64_t seed, uint64_t uid) {
    U64x4 o = philox4x64_10(uid, 0ull, (uint64_t)RNG_INIT, 0ull, seed, 0ull);
    return -log(u01(o.a));
}

// ------------------------------------------------------------------------
// Real-type helpers: the FP64 form and the FP32 precision form.
// ------------------------------------------------------------------------
// The FP64 form uses the correctly rounded library functions.  The FP32
// precision form uses the hardware's single-precision square root,
// reciprocal, base-2 logarithm and exponential (V_SQRT_F32, V_RCP_F32,
// V_LOG_F32, V_EXP_F32, each within about one ulp for the normal arguments
// met here); their error is far below the form's 1e-5 bar on the momenta.
template <typename R> struct Math;
template <> struct Math<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double log_(double x) { return log(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div_(double a, double b) { return a / b; }
};
template <> struct Math<float> {
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float log_(float x) {
        return __builtin_amdgcn_logf(x) * 0.693147180559945309f;              // ln 2
    }
    static __device__ __forceinline__ float exp_(float x) {
        return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);              // log2 e
    }
    static __device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};

// ------------------------------------------------------------------------
// Tables in device memory (FP64 and FP32 copies) and their layout.
// ------------------------------------------------------------------------
struct TablesDev {
    const double *ln_hrad, *ln_g, *emit_q, *pair_lnh, *pair_q;
    const float *ln_hrad_f, *ln_g_f, *emit_q_f, *pair_lnh_f, *pair_q_f;
    int e_n_chi, e_n_q, p_n_chi, p_n_q;
    double e_chi_min, e_inv_chi_min, e_h0;   // first emission node, 1/chi there, h_rad there
    double e_lnchi0, e_inv_dlnchi, e_logit_max, e_inv_dt;
    double p_chi_min, p_lnchi0, p_inv_dlnchi, p_logit_max, p_inv_dt;
    // spline form of the quantile tables (null when bilinear): per node the
    // value and its curvatures f_tt, f_cc, f_cctt; h^2/6 of both node spacings
    const double *emit_qs, *pair_qs;
    const float *emit_qs_f, *pair_qs_f;
    double e_ht26, e_hc26, p_ht26, p_hc26;
};

template <typename R> __device__ __forceinline__ const R *emit_q_ptr(const TablesDev &t);
template <> __device__ __forceinline__ const double *emit_q_ptr<double>(const TablesDev &t) { return t.emit_q; }
template <> __device__ __forceinline__ const float *emit_q_ptr<float>(const TablesDev &t) { return t.emit_q_f; }
template <typename R> __device__ __forceinline__ const R *pair_q_ptr(const TablesDev &t);
template <> __device__ __forceinline__ const double *pair_q_ptr<double>(const TablesDev &t) { return t.pair_q; }
template <> __device__ __forceinline__ const float *pair_q_ptr<float>(const TablesDev &t) { return t.pair_q_f; }
template <typename R> __device__ __forceinline__ const R *emit_qs_ptr(const TablesDev &t);
template <> __device__ __forceinline__ const double *emit_qs_ptr<double>(const TablesDev &t) { return t.emit_qs; }
template <> __device__ __forceinline__ const float *emit_qs_ptr<float>(const TablesDev &t) { return t.emit_qs_f; }
template <typename R> __device__ __forceinline__ const R *pair_qs_ptr(const TablesDev &t);
template <> __device__ __forceinline__ const double *pair_qs_ptr<double>(const TablesDev &t) { return t.pair_qs; }
template <> __device__ __forceinline__ const float *pair_qs_ptr<float>(const TablesDev &t) { return t.pair_qs_f; }
template <typename R> __device__ __forceinline__ const R *rate_ptr(const TablesDev &t, int which);
template <> __device__ __forceinline__ const double *rate_ptr<double>(const TablesDev &t, int w) {
    return w == 0 ? t.ln_hrad : (w == 1 ? t.ln_g : t.pair_lnh);
}
template <> __device__ __forceinline__ const float *rate_ptr<float>(const TablesDev &t, int w) {
    return w == 0 ? t.ln_hrad_f : (w == 1 ? t.ln_g_f : t.pair_lnh_f);
}

// Linear interpolation in (ln chi, ln rate) from a table staged in LDS; the
// end segments are extended outside the node range; *above is set when chi
// lies beyond the last node.
template <typename R>
__device__ __forceinline__ R lerp_rate(const R *lds, int n, R lnchi0, R inv_d, R lnchi, bool &above) {
    R u = (lnchi - lnchi0) * inv_d;
    int i;
    if (!(u >= R(0))) i = 0;                       // below the table, or NaN
    else if (u >= R(n - 1)) { i = n - 2; above = true; }
    else i = (int)u;
    const R w = u - (R)i;
    const R a = lds[i], b = lds[i + 1];
    return a + w * (b - a);
}

// Emission rate h_rad of Eq. 2 at chi_e from the table staged in LDS.  Below
// the first node the rate follows the classical law, proportional to chi,
// equal to the node value there; *above is set beyond the last node.
template <typename R>
__device__ __forceinline__ R h_rad_at(const R *s_lh, const TablesDev &tb, R lnchi0, R inv_d, R chi, bool &above) {
    if (chi < (R)tb.e_chi_min) return (R)tb.e_h0 * (chi * (R)tb.e_inv_chi_min);
    return Math<R>::exp_(lerp_rate<R>(s_lh, tb.e_n_chi, lnchi0, inv_d, Math<R>::log_(chi), above));
}

// g(chi_e) = P_rad / P_classical of Eq. 5 from the table staged in LDS.  Below
// the first node ln g is proportional to chi (the first-order law
// g = 1 - (55 sqrt 3/16) chi), equal to the node value there, so that g -> 1
// and P_rad tends to the classical Larmor power.
template <typename R>
__device__ __forceinline__ R g_at(const R *s_lg, const TablesDev &tb, R lnchi0, R inv_d, R chi) {
    if (chi < (R)tb.e_chi_min) return Math<R>::exp_(s_lg[0] * (chi * (R)tb.e_inv_chi_min));
    bool above = false;
    return Math<R>::exp_(lerp_rate<R>(s_lg, tb.e_n_chi, lnchi0, inv_d, Math<R>::log_(chi), above));
}

// One cubic segment of a natural spline at fraction z of its step:
// (1-z) f0 + z f1 + (h^2/6) [((1-z)^3 - (1-z)) m0 + (z^3 - z) m1].
template <typename R>
__device__ __forceinline__ R spline_seg(R f0, R f1, R m0, R m1, R z, R h26) {
    const R a = R(1) - z;
    return a * f0 + z * f1 + ((a * a - R(1)) * a * m0 + (z * z - R(1)) * z * m1) * h26;
}

// Lookup in (ln chi, logit r) of a quantile table in global memory
// (L2-resident); chi is clamped to the node range.  The logit of r is taken
// in FP64 so that the extreme levels keep their resolution in both forms.
// With qs null: bilinear in the node cell.  With qs (four values per node:
// f, f_tt, f_cc, f_cctt): the tensor-product natural cubic spline, first
// along t in the cell's two rows (for f and for f_cc), then along ln chi.
template <typename R>
__device__ __forceinline__ R quantile(const R *q, const R *qs, R ht26, R hc26, int n_chi, int n_q, R lnchi0,
                                      R inv_d, double logit_max, double inv_dt, R lnchi, double r) {
    R u = (lnchi - lnchi0) * inv_d;
    if (!(u > R(0))) u = R(0);
    if (u > R(n_chi - 1)) u = R(n_chi - 1);
    int i = (int)u;
    if (i > n_chi - 2) i = n_chi - 2;
    const R w = u - (R)i;
    double t = log(r) - log(1.0 - r);
    if (!(t > -logit_max)) t = -logit_max;
    if (t > logit_max) t = logit_max;
    const double v = (t + logit_max) * inv_dt;
    int j = (int)v;
    if (j > n_q - 2) j = n_q - 2;
    const R z = (R)(v - (double)j);
    if (qs) {
        const R *n0 = qs + 4 * ((size_t)i * n_q + j), *n1 = n0 + 4 * (size_t)n_q;
        const R f0 = spline_seg<R>(n0[0], n0[4], n0[1], n0[5], z, ht26);
        const R f1 = spline_seg<R>(n1[0], n1[4], n1[1], n1[5], z, ht26);
        const R c0 = spline_seg<R>(n0[2], n0[6], n0[3], n0[7], z, ht26);
        const R c1 = spline_seg<R>(n1[2], n1[6], n1[3], n1[7], z, ht26);
        return spline_seg<R>(f0, f1, c0, c1, w, hc26);
    }
    const R *r0 = q + (size_t)i * n_q + j;
    const R *r1 = r0 + n_q;
    const R a = r0[0] + z * (r0[1] - r0[0]);
    const R b = r1[0] + z * (r1[1] - r1[0]);
    return a + w * (b - a);
}

// ------------------------------------------------------------------------
// Quantum parameter, Eq. 1 in covariant form:
//   chi = sqrt((g E + p x B)^2 - (p.E)^2) / E_s
// (g = gamma, p = u for leptons; g = |k|, p = k for photons).
// ------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R chi_of(R es_inv, R g, R px, R py, R pz, const R E[3], const R B[3]) {
    const R fx = g * E[0] + (py * B[2] - pz * B[1]);
    const R fy = g * E[1] + (pz * B[0] - px * B[2]);
    const R fz = g * E[2] + (px * B[1] - py * B[0]);
    const R pe = px * E[0] + py * E[1] + pz * E[2];
    const R q = (fx * fx + fy * fy + fz * fz) - pe * pe;
    return (q > R(0) ? Math<R>::sqrt_(q) : R(0)) * es_inv;
}

// ------------------------------------------------------------------------
// Wave-level scans (wave64).
// ------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// exclusive prefix of a 0/1 flag across the wave, and the wave total
__device__ __forceinline__ uint32_t ballot_excl(bool flag, uint32_t &total) {
    const uint64_t m = __ballot(flag);
    total = (uint32_t)__popcll(m);
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t &total) {
    const int lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

// Sum over the wave, on every lane: row sums through DPP (quad permutations,
// row rotations), then the four rows.  The wave must be fully active.
// (The DPP patterns used below read a valid source lane for every lane, so
// the moves need no prior value in their destination.)
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_mov_dpp(x, 0xb1, 0xf, 0xf, false);     // quad_perm 1,0,3,2
    x += __builtin_amdgcn_mov_dpp(x, 0x4e, 0xf, 0xf, false);     // quad_perm 2,3,0,1
    x += __builtin_amdgcn_mov_dpp(x, 0x124, 0xf, 0xf, false);    // row_ror 4
    x += __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, false);    // row_ror 8
    return (uint32_t)__builtin_amdgcn_readlane(x, 0) + (uint32_t)__builtin_amdgcn_readlane(x, 16) +
           (uint32_t)__builtin_amdgcn_readlane(x, 32) + (uint32_t)__builtin_amdgcn_readlane(x, 48);
}

// Sum over the wave of a double, on every lane, in a fixed tree order: row
// sums through DPP on both halves of the value, then the four rows in order.
// The wave must be fully active.
__device__ __forceinline__ double wave_sum_f64_dpp(double v) {
    auto step = [](double x, auto ctrl) {
        const uint64_t b = __builtin_bit_cast(uint64_t, x);
        const int lo = __builtin_amdgcn_mov_dpp((int)b, decltype(ctrl)::value, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), decltype(ctrl)::value, 0xf, 0xf, false);
        return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    };
    v += step(v, std::integral_constant<int, 0xb1>{});    // quad_perm 1,0,3,2
    v += step(v, std::integral_constant<int, 0x4e>{});    // quad_perm 2,3,0,1
    v += step(v, std::integral_constant<int, 0x124>{});   // row_ror 4
    v += step(v, std::integral_constant<int, 0x128>{});   // row_ror 8
    auto lane_value = [](double x, int l) {
        const uint64_t b = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)b, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(b >> 32), l);
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    };
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sums over the wave of two doubles, a and b, through one DPP chain: the first
// step adds lane pairs (l, l xor 1) so that even lanes hold pair sums of a and
// odd lanes pair sums of b; every later step combines lanes of equal parity.
// Each sum is formed in the order of wave_sum_f64_dpp (addition commutes), so
// the results are those of two separate calls.  The wave must be fully active.
__device__ __forceinline__ void wave_sum2_f64_dpp(double a, double b, double &sa, double &sb) {
    auto mov = [](double x, auto ctrl) {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const int lo = __builtin_amdgcn_mov_dpp((int)u, decltype(ctrl)::value, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), decltype(ctrl)::value, 0xf, 0xf, false);
        return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    };
    const bool odd = (lane_id() & 1) != 0;
    double v = (odd ? b : a) + mov(odd ? a : b, std::integral_constant<int, 0xb1>{});   // quad_perm 1,0,3,2
    v += mov(v, std::integral_constant<int, 0x4e>{});                                   // quad_perm 2,3,0,1
    v += mov(v, std::integral_constant<int, 0x124>{});                                  // row_ror 4
    v += mov(v, std::integral_constant<int, 0x128>{});                                  // row_ror 8
    auto lane_value = [](double x, int l) {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)u, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(u >> 32), l);
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    };
    sa = (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
    sb = (lane_value(v, 1) + lane_value(v, 17)) + (lane_value(v, 33) + lane_value(v, 49));
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// ------------------------------------------------------------------------
// Decoupled look-back (Merrill & Garland, 2016) over tiles taken in ticket
// order, for two append streams at once.  Each tile publishes its aggregate
// and later its inclusive prefix as 64-bit words (launch epoch << 32 | value),
// so a stale word from an earlier launch never matches and the arrays need
// no clearing.  One wave scans 64 predecessors per round.
// ------------------------------------------------------------------------
struct LookBack {
    uint64_t *agg0, *agg1, *inc0, *inc1;
};

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint32_t v) {
    return ((uint64_t)epoch << 32) | (uint64_t)v;
}

// Called by all 64 lanes of one wave; returns the exclusive prefixes.
__device__ __forceinline__ void lookback2(const LookBack &lb, int64_t tile, uint32_t epoch,
                                          uint32_t a0, uint32_t a1, uint32_t &p0, uint32_t &p1) {
    const int lane = lane_id();
    if (tile == 0) {
        if (lane == 0) { lb_store(lb.inc0, lb_pack(epoch, a0)); lb_store(lb.inc1, lb_pack(epoch, a1)); }
        p0 = 0; p1 = 0;
        return;
    }
    if (lane == 0) { lb_store(lb.agg0 + tile, lb_pack(epoch, a0)); lb_store(lb.agg1 + tile, lb_pack(epoch, a1)); }
    uint32_t s0 = 0, s1 = 0;
    int64_t top = tile - 1;
    for (;;) {
        const int64_t idx = top - lane;
        int state = 2;            // 0 not ready, 1 aggregate, 2 inclusive (or before tile 0)
        uint32_t v0 = 0, v1 = 0;
        if (idx >= 0) {
            const uint64_t i0 = lb_load(lb.inc0 + idx), i1 = lb_load(lb.inc1 + idx);
            if ((uint32_t)(i0 >> 32) == epoch && (uint32_t)(i1 >> 32) == epoch) {
                v0 = (uint32_t)i0; v1 = (uint32_t)i1;
            } else {
                const uint64_t g0 = lb_load(lb.agg0 + idx), g1 = lb_load(lb.agg1 + idx);
                if ((uint32_t)(g0 >> 32) == epoch && (uint32_t)(g1 >> 32) == epoch) {
                    state = 1; v0 = (uint32_t)g0; v1 = (uint32_t)g1;
                } else {
                    state = 0;
                }
            }
        }
        const uint64_t incl = __ballot(state == 2);
        const uint64_t wait = __ballot(state == 0);
        const int first = incl ? (__ffsll((unsigned long long)incl) - 1) : kWave;
        const uint64_t need = (first >= kWave - 1) ? ~0ull : ((2ull << first) - 1ull);
        if (wait & need) { __builtin_amdgcn_s_sleep(1); continue; }
        const bool take = lane <= first;
        s0 += wave_sum_u32(take ? v0 : 0u);
        s1 += wave_sum_u32(take ? v1 : 0u);
        if (first < kWave) break;
        top -= kWave;
    }
    if (lane == 0) { lb_store(lb.inc0 + tile, lb_pack(epoch, s0 + a0)); lb_store(lb.inc1 + tile, lb_pack(epoch, s1 + a1)); }
    p0 = s0; p1 = s1;
}

// Inclusive total of the last tile, spun for by the launch's final requester.
__device__ __forceinline__ void lb_wait_inclusive(const LookBack &lb, int64_t tile, uint32_t epoch,
                                                  uint32_t &t0, uint32_t &t1) {
    uint64_t w0, w1;
    do { w0 = lb_load(lb.inc0 + tile); } while ((uint32_t)(w0 >> 32) != epoch);
    do { w1 = lb_load(lb.inc1 + tile); } while ((uint32_t)(w1 >> 32) != epoch);
    t0 = (uint32_t)w0;
    t1 = (uint32_t)w1;
}

// Block-wide exclusive scan of two small counts per thread (block <= 1024).
// s_wave must hold 2*kMaxWaves words; returns the block totals.
__device__ __forceinline__ void block_scan2(uint32_t c0, uint32_t c1, uint32_t &e0, uint32_t &e1,
                                            uint32_t &tot0, uint32_t &tot1, uint32_t *s_wave) {
    uint32_t w0, w1;
    const uint32_t x0 = wave_excl_scan(c0, w0);
    const uint32_t x1 = wave_excl_scan(c1, w1);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane_id() == 0) { s_wave[wid] = w0; s_wave[kMaxWaves + wid] = w1; }
    __syncthreads();
    uint32_t o0 = 0, o1 = 0, t0 = 0, t1 = 0;
    for (int k = 0; k < nw; ++k) {
        const uint32_t a = s_wave[k], b = s_wave[kMaxWaves + k];
        if (k < wid) { o0 += a; o1 += b; }
        t0 += a; t1 += b;
    }
    e0 = o0 + x0; e1 = o1 + x1;
    tot0 = t0; tot1 = t1;
}

// Exclusive rank of a 0/1 flag and the block totals of the flag and of two
// counts (block <= 256 threads); s_wave holds 3*kMaxWaves words.
__device__ __forceinline__ void block_rank3(bool f, uint32_t c0, uint32_t c1, uint32_t &rank,
                                            uint32_t &tf, uint32_t &t0, uint32_t &t1, uint32_t *s_wave) {
    uint32_t wf;
    const uint32_t x = ballot_excl(f, wf);
    const uint32_t w0 = wave_sum_u32(c0), w1 = wave_sum_u32(c1);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane_id() == 0) { s_wave[wid] = wf; s_wave[kMaxWaves + wid] = w0; s_wave[2 * kMaxWaves + wid] = w1; }
    __syncthreads();
    uint32_t o = 0, a = 0, b = 0, c = 0;
    for (int k = 0; k < nw; ++k) {
        const uint32_t v = s_wave[k];
        if (k < wid) o += v;
        a += v;
        b += s_wave[kMaxWaves + k];
        c += s_wave[2 * kMaxWaves + k];
    }
    rank = o + x;
    tf = a; t0 = b; t1 = c;
}

// Same for 0/1 flags, using the wave ballot.
__device__ __forceinline__ void block_scan_flag(bool f, uint32_t &e, uint32_t &tot, uint32_t *s_wave) {
    uint32_t w;
    const uint32_t x = ballot_excl(f, w);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane_id() == 0) s_wave[wid] = w;
    __syncthreads();
    uint32_t o = 0, t = 0;
    for (int k = 0; k < nw; ++k) {
        const uint32_t a = s_wave[k];
        if (k < wid) o += a;
        t += a;
    }
    e = o + x;
    tot = t;
}

}  // namespace qed
