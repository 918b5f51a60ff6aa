// qed_tables.cpp -- FP64 host construction of the rate and quantile tables
// used by the QED step (Lobet et al., arXiv:1311.1107, Eqs. 2, 3, 5, 6, 7).
//
// Quantities (chi = chi_e for emission, chi_gamma for pairs):
//   emission spectrum in xi = chi_gamma/chi_e (Eq. 2, positive form):
//     S_e(xi) = (2 + xi^2/(1-xi)) K_{2/3}(d) - Int_d^inf K_{1/3},  d = 2 xi/(3 chi (1-xi))
//   h_rad = (1/(pi sqrt3)) Int_0^1 S_e,  g = (sqrt3/(2 pi chi^2)) Int_0^1 xi S_e,
//   pair spectrum in eta = chi_-/chi_gamma (Eq. 3 with y = 1/(3 chi eta(1-eta))):
//     S_p(eta) = Int_d^inf K_{1/3} + (1/(eta(1-eta)) - 2) K_{2/3}(d),  d = 2/(3 chi eta(1-eta))
//   h_pair = (1/(pi sqrt3)) Int_0^1 S_p,
//   quantiles: ln xi (emission) and logit eta (pair) where the normalised
//   running integral reaches r_k = 1/(1+exp(-t_k)).
//
// Method: the Bessel functions come from K_nu(x) = Int_0^inf exp(-x cosh t)
// cosh(nu t) dt and Int_x^inf K_nu = Int_0^inf exp(-x cosh t) cosh(nu t)/cosh t dt,
// integrated by 24-point Gauss-Legendre on t-panels (scaled by e^x); the outer
// integrals use the logistic variable v (xi = 1/(1+e^-v)) with 16-point
// Gauss-Legendre panels; quantiles are found by Newton iteration bracketed by
// the panel running sums.  Work is spread over host threads, one chi node at
// a time.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

namespace qedtab {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Gauss-Legendre nodes on [-1,1] from the three-term recurrence, polished by Newton.
struct Rule {
    std::vector<double> x, w;
    explicit Rule(int n) : x(n), w(n) {
        for (int i = 0; i < n; ++i) {
            // Tricomi's initial approximation of the i-th root
            double th = kPi * (4.0 * i + 3.0) / (4.0 * n + 2.0);
            double z = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
            double pd = 1.0;
            for (int it = 0; it < 60; ++it) {
                double pm = 1.0, p = z;
                for (int k = 2; k <= n; ++k) {
                    double pk = ((2 * k - 1) * z * p - (k - 1) * pm) / k;
                    pm = p;
                    p = pk;
                }
                pd = n * (pm - z * p) / (1.0 - z * z);
                double dz = p / pd;
                z -= dz;
                if (std::fabs(dz) <= 1e-17) break;
            }
            double pm = 1.0, p = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2 * k - 1) * z * p - (k - 1) * pm) / k;
                pm = p;
                p = pk;
            }
            pd = n * (pm - z * p) / (1.0 - z * z);
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * pd * pd);
        }
    }
};

const Rule &rule24() { static const Rule r(24); return r; }
const Rule &rule16() { static const Rule r(16); return r; }

// e^x K_{2/3}(x) and e^x Int_x^inf K_{1/3}, both from one pass over t.
// The integrand exp(-2x sinh^2(t/2)) decays past t ~ 2 asinh(sqrt(40/x)) and
// grows like e^{2t/3} before x cosh t ~ 1.  For x <= 9 unit-width t-panels
// with 16 nodes each are used, their node quantities tabulated once; for
// larger x the bump has width ~1/sqrt(x) and panels of width 1.5/sqrt(x).
struct TNodes {
    static constexpr int kPanels = 170;
    std::vector<double> c, wk, wi;   // 2 sinh^2(t/2), w cosh(2t/3), w cosh(t/3)/cosh t
    TNodes() {
        const Rule &R = rule16();
        const int m = (int)R.x.size();
        c.resize(kPanels * m); wk.resize(kPanels * m); wi.resize(kPanels * m);
        for (int p = 0; p < kPanels; ++p)
            for (int j = 0; j < m; ++j) {
                double t = p + 0.5 + 0.5 * R.x[j];
                double sh = std::sinh(0.5 * t);
                c[p * m + j] = 2.0 * sh * sh;
                wk[p * m + j] = 0.5 * R.w[j] * std::cosh(2.0 * t / 3.0);
                wi[p * m + j] = 0.5 * R.w[j] * std::cosh(t / 3.0) / std::cosh(t);
            }
    }
};

const TNodes &tnodes() { static const TNodes n; return n; }

void bessel_pair_scaled(double x, double &k23, double &ki13) {
    double sk = 0.0, si = 0.0;
    if (x <= 9.0) {
        const TNodes &N = tnodes();
        const int m = (int)rule16().x.size();
        for (int p = 0; p < TNodes::kPanels; ++p) {
            for (int j = p * m; j < (p + 1) * m; ++j) {
                double e = std::exp(-x * N.c[j]);
                sk += e * N.wk[j];
                si += e * N.wi[j];
            }
            double shb = std::sinh(0.5 * (p + 1.0));
            if (2.0 * x * shb * shb > 45.0 + (p + 1.0)) break;
        }
        k23 = sk;
        ki13 = si;
        return;
    }
    const Rule &R = rule24();
    double width = 1.5 / std::sqrt(x);
    for (int p = 0; p < 100000; ++p) {
        double a = p * width, b = a + width;
        double half = 0.5 * width, mid = a + half;
        double pk = 0.0, pi = 0.0;
        for (size_t m = 0; m < R.x.size(); ++m) {
            double t = mid + half * R.x[m];
            double sh = std::sinh(0.5 * t);
            double e = std::exp(-2.0 * x * sh * sh);
            pk += R.w[m] * e * std::cosh(2.0 * t / 3.0);
            pi += R.w[m] * e * std::cosh(t / 3.0) / std::cosh(t);
        }
        sk += pk * half;
        si += pi * half;
        double shb = std::sinh(0.5 * b);
        if (2.0 * x * shb * shb > 45.0 + b) break;
    }
    k23 = sk;
    ki13 = si;
}

// emission integrand in v: S_e(xi(v)) dxi/dv, and the pair integrand in v
// scaled by exp(8/(3chi)).
double emit_dv(double chi, double v) {
    double ev = std::exp(v);
    double xi = std::isinf(ev) ? 1.0 : ev / (1.0 + ev);
    double jac = std::isinf(ev) ? 0.0 : ev / ((1.0 + ev) * (1.0 + ev));
    double d = 2.0 * ev / (3.0 * chi);
    if (!(d < 720.0)) return 0.0;
    double k23, ki13;
    bessel_pair_scaled(d, k23, ki13);
    return std::exp(-d) * ((2.0 + xi * ev) * k23 - ki13) * jac;
}

double pair_dv(double chi, double v) {
    double ch = std::cosh(0.5 * v), sh = std::sinh(0.5 * v);
    double inv_e = 4.0 * ch * ch;                    // 1/(eta (1-eta))
    double d = inv_e * 2.0 / (3.0 * chi);
    double over = 8.0 * sh * sh / (3.0 * chi);       // d - 8/(3chi)
    if (!(over < 720.0)) return 0.0;
    double k23, ki13;
    bessel_pair_scaled(d, k23, ki13);
    return std::exp(-over) * (ki13 + (inv_e - 2.0) * k23) / inv_e;
}

typedef double (*Integrand)(double, double);

double panel(Integrand f, double chi, double a, double b, bool weight_xi) {
    const Rule &R = rule16();
    double half = 0.5 * (b - a), mid = 0.5 * (a + b), s = 0.0;
    for (size_t m = 0; m < R.x.size(); ++m) {
        double v = mid + half * R.x[m];
        double y = f(chi, v);
        if (weight_xi) y /= (1.0 + std::exp(-v));
        s += R.w[m] * y;
    }
    return s * half;
}

// Emission mass left of the first edge v0: as v -> -inf the integrand tends
// to c e^{v/3} (xi ~ e^v, K_{2/3}(d) ~ Gamma(2/3) 2^{-1/3} d^{-2/3}), with
// relative corrections O(e^{2v/3}), so the tail is 3 emit_dv(v0).
double left_tail(Integrand f, double chi, double v0) {
    return f == emit_dv ? 3.0 * emit_dv(chi, v0) : 0.0;
}

std::vector<double> emit_edges(double chi) {
    std::vector<double> e;
    double top = std::log(chi * 1100.0) + 0.7;
    for (double v = -110.0; v < -24.0; v += 2.5) e.push_back(v);
    int n = (int)std::ceil((top + 24.0) / 0.4);
    for (int k = 0; k <= n; ++k) e.push_back(-24.0 + (top + 24.0) * k / n);
    return e;
}

std::vector<double> pair_edges(double chi) {
    double half = std::acosh(1.0 + 560.0 * chi) + 0.3;
    int n = std::max(10, (int)std::ceil(2.0 * half / 0.2));
    std::vector<double> e(n + 1);
    for (int k = 0; k <= n; ++k) e[k] = -half + 2.0 * half * k / n;
    return e;
}

// Quantiles of the normalised running integral of f at the logit levels.
void quantiles(Integrand f, double chi, const std::vector<double> &edge, int n_q,
               double logit_max, double *out_v) {
    int np = (int)edge.size() - 1;
    std::vector<double> part(np), below(np + 1), above(np + 1);
    for (int k = 0; k < np; ++k) part[k] = panel(f, chi, edge[k], edge[k + 1], false);
    below[0] = left_tail(f, chi, edge[0]);
    for (int k = 0; k < np; ++k) below[k + 1] = below[k] + part[k];
    above[np] = 0.0;
    for (int k = np - 1; k >= 0; --k) above[k] = above[k + 1] + part[k];
    above[0] += below[0];
    for (int q = 0; q < n_q; ++q) {
        double t = -logit_max + 2.0 * logit_max * q / (n_q - 1);
        bool hi_side = t > 0.0;
        // target mass measured from the nearer end, for relative accuracy in the tails
        double goal = hi_side ? above[0] / (1.0 + std::exp(t)) : below[np] / (1.0 + std::exp(-t));
        int k = 0;
        if (!hi_side) {
            while (k < np - 1 && below[k + 1] <= goal) ++k;
        } else {
            k = np - 1;
            while (k > 0 && above[k] <= goal) --k;
        }
        double a = edge[k], b = edge[k + 1];
        // mass from the near end to v, minus the goal: increasing (low side) or decreasing
        auto resid = [&](double v) {
            return hi_side ? above[k + 1] + panel(f, chi, v, b, false) - goal
                           : below[k] + panel(f, chi, a, v, false) - goal;
        };
        double lo = a, hi = b;
        double frac = hi_side ? (goal - above[k + 1]) / part[k] : (goal - below[k]) / part[k];
        double v = hi_side ? b - frac * (b - a) : a + frac * (b - a);
        if (!(v > lo && v < hi)) v = 0.5 * (lo + hi);
        for (int it = 0; it < 80; ++it) {
            double r = resid(v);
            bool past = hi_side ? (r < 0.0) : (r > 0.0);
            if (past) hi = v; else lo = v;
            double slope = hi_side ? -f(chi, v) : f(chi, v);
            double nv = (slope != 0.0) ? v - r / slope : 0.5 * (lo + hi);
            if (!(nv > lo && nv < hi)) nv = 0.5 * (lo + hi);
            double step = std::fabs(nv - v);
            v = nv;
            if (step <= 2e-16 * (1.0 + std::fabs(v)) || hi - lo <= 2e-16 * (1.0 + std::fabs(v))) break;
        }
        out_v[q] = v;
    }
}

}  // namespace

// Returns 0 on success.
int build_tables(double e_chi_min, double e_chi_max, int e_n_chi, int e_n_q, double e_logit,
                 double p_chi_min, double p_chi_max, int p_n_chi, int p_n_q, double p_logit,
                 double *ln_hrad, double *ln_g, double *emit_q, double *pair_lnh, double *pair_q) {
    rule24();
    rule16();
    tnodes();
    const double l0e = std::log(e_chi_min), l1e = std::log(e_chi_max);
    const double l0p = std::log(p_chi_min), l1p = std::log(p_chi_max);
    const int jobs = e_n_chi + p_n_chi;
    std::atomic<int> next(0);
    auto worker = [&]() {
        for (;;) {
            int j = next.fetch_add(1);
            if (j >= jobs) return;
            if (j < e_n_chi) {
                double chi = std::exp(l0e + (l1e - l0e) * j / (e_n_chi - 1));
                std::vector<double> edge = emit_edges(chi);
                double tot = left_tail(emit_dv, chi, edge[0]), mom = 0.0;
                for (size_t k = 0; k + 1 < edge.size(); ++k) {
                    tot += panel(emit_dv, chi, edge[k], edge[k + 1], false);
                    mom += panel(emit_dv, chi, edge[k], edge[k + 1], true);
                }
                ln_hrad[j] = std::log(tot / (kPi * std::sqrt(3.0)));
                ln_g[j] = std::log(std::sqrt(3.0) * mom / (2.0 * kPi * chi * chi));
                double *row = emit_q + (size_t)j * e_n_q;
                quantiles(emit_dv, chi, edge, e_n_q, e_logit, row);
                for (int q = 0; q < e_n_q; ++q) row[q] = -std::log1p(std::exp(-row[q]));
            } else {
                int i = j - e_n_chi;
                double chi = std::exp(l0p + (l1p - l0p) * i / (p_n_chi - 1));
                std::vector<double> edge = pair_edges(chi);
                double tot = 0.0;
                for (size_t k = 0; k + 1 < edge.size(); ++k) tot += panel(pair_dv, chi, edge[k], edge[k + 1], false);
                pair_lnh[i] = std::log(tot / (kPi * std::sqrt(3.0)));
                quantiles(pair_dv, chi, edge, p_n_q, p_logit, pair_q + (size_t)i * p_n_q);
            }
        }
    };
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned k = 1; k < nt; ++k) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    for (int i = 0; i < e_n_chi; ++i)
        if (!std::isfinite(ln_hrad[i]) || !std::isfinite(ln_g[i])) return 1;
    for (int i = 0; i < p_n_chi; ++i)
        if (!std::isfinite(pair_lnh[i])) return 1;
    return 0;
}

// Curvature of the natural cubic spline (zero second derivative at both
// ends) through n values spaced h apart, read with stride `step`: the
// interior second derivatives solve the tridiagonal system
//   c[k-1] + 4 c[k] + c[k+1] = 6 (y[k-1] - 2 y[k] + y[k+1]) / h^2.
// Gaussian elimination down the band, then back substitution.
static void spline_curvature(const double *y, size_t step, int n, double h, double *c, size_t cstep) {
    std::vector<double> diag(n, 4.0), rhs(n, 0.0);
    c[0] = 0.0;
    c[(size_t)(n - 1) * cstep] = 0.0;
    if (n < 3) return;
    for (int k = 1; k < n - 1; ++k)
        rhs[k] = 6.0 * (y[(k - 1) * step] - 2.0 * y[k * step] + y[(k + 1) * step]) / (h * h);
    for (int k = 2; k < n - 1; ++k) {          // eliminate the sub-diagonal (all ones)
        const double f = 1.0 / diag[k - 1];
        diag[k] -= f;
        rhs[k] -= f * rhs[k - 1];
    }
    double next = 0.0;
    for (int k = n - 2; k >= 1; --k) {
        next = (rhs[k] - next) / diag[k];
        c[k * cstep] = next;
    }
}

void spline_quads(const double *q, int n_chi, int n_q, double h_c, double h_t, double *quad) {
    const size_t N = (size_t)n_chi * n_q;
    std::vector<double> ctt(N), ccc(N), cccc(N);
    for (int i = 0; i < n_chi; ++i) spline_curvature(q + (size_t)i * n_q, 1, n_q, h_t, &ctt[(size_t)i * n_q], 1);
    for (int j = 0; j < n_q; ++j) spline_curvature(q + j, n_q, n_chi, h_c, &ccc[j], n_q);
    for (int i = 0; i < n_chi; ++i)
        spline_curvature(&ccc[(size_t)i * n_q], 1, n_q, h_t, &cccc[(size_t)i * n_q], 1);
    for (size_t k = 0; k < N; ++k) {
        quad[4 * k + 0] = q[k];
        quad[4 * k + 1] = ctt[k];
        quad[4 * k + 2] = ccc[k];
        quad[4 * k + 3] = cccc[k];
    }
}

}  // namespace qedtab
