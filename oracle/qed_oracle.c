/*
 * qed_oracle.c -- CPU oracle for the per-particle radiation-and-QED step of
 * Lobet et al. (arXiv:1311.1107).  TEST INFRASTRUCTURE: used only by tests,
 * by the smoke check and by the benchmark's CPU-baseline leg; never by the
 * product.  Everything is FP64 and serial in particle-index order, written to
 * be checked against the paper by eye rather than to be fast.
 *
 * Readings of passages the paper leaves garbled or open are marked READING.
 */
#include "qed_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ======================================================================== *
 * 1. Constants (Sec. 2: E_s after Eq. 1, alpha_f and tau_c after Eq. 2,
 *    tau_0 after Eq. 4).  CODATA 2018 values.
 * ======================================================================== */
void or_units_init(double lambda_m, or_units *u)
{
    const double c    = 299792458.0;
    const double e    = 1.602176634e-19;
    const double h    = 6.62607015e-34;
    const double hbar = h / (2.0 * M_PI);
    const double m    = 9.1093837015e-31;
    const double eps0 = 8.8541878128e-12;

    u->lambda  = lambda_m;
    u->omega_r = 2.0 * M_PI * c / lambda_m;
    u->alpha_f = e * e / (4.0 * M_PI * eps0 * hbar * c);
    u->E_s     = m * m * c * c * c / (e * hbar);            /* after Eq. 1 */
    u->B_s     = u->E_s / c;
    /* READING: the paper calls tau_c = hbar/(m c^2) a "Compton length"; the
     * prefactor alpha_f/(tau_c gamma^2) of Eq. 2 is a rate, so tau_c is the
     * Compton time. */
    u->tau_c   = hbar / (m * c * c);
    u->tau_0   = 2.0 * e * e / (12.0 * M_PI * eps0 * m * c * c * c);  /* after Eq. 4 */
    u->E_ref   = m * c * u->omega_r / e;
    u->B_ref   = m * u->omega_r / e;
    u->Es_hat  = u->E_s / u->E_ref;
    u->A_hat   = u->alpha_f / (u->tau_c * u->omega_r);
    u->tau0_hat = u->tau_0 * u->omega_r;
}

/* ======================================================================== *
 * 2. Modified Bessel functions used by Eqs. 2-3.
 *
 *   K_nu(x)          = int_0^inf exp(-x cosh t) cosh(nu t) dt
 *   int_x^inf K_nu   = int_0^inf exp(-x cosh t) cosh(nu t)/cosh t dt
 *
 * (the second by exchanging the order of integration).  Both integrands are
 * even and analytic in a strip about the real t axis, so the trapezoidal rule
 * with step h converges like exp(-2 pi d/h).  We return the values scaled by
 * e^x, i.e. with exp(-x (cosh t - 1)) = exp(-2 x sinh^2(t/2)) in the
 * integrand, which keeps them representable for large x.
 * ======================================================================== */
#define BK_H      0.125
#define BK_NMAX   1400

static double bk_c[BK_NMAX];       /* 2 sinh^2(t_k/2) = cosh t_k - 1 */
static double bk_t[BK_NMAX];
static double bk_cosh[BK_NMAX];
static int bk_ready = 0;

static void bk_init(void)
{
    if (bk_ready) return;
    for (int k = 0; k < BK_NMAX; ++k) {
        double t = k * BK_H;
        double sh = sinh(0.5 * t);
        bk_t[k] = t;
        bk_c[k] = 2.0 * sh * sh;
        bk_cosh[k] = cosh(t);
    }
    bk_ready = 1;
}

/* e^x K_nu(x) (kind 0) or e^x int_x^inf K_nu (kind 1) */
static double bessel_scaled(double nu, double x, int kind)
{
    if (x <= 16.0) {
        double sum = 0.0;
        for (int k = 0; k < BK_NMAX; ++k) {
            double t = bk_t[k];
            double ex = x * bk_c[k];
            double term = exp(-ex) * cosh(nu * t);
            if (kind) term /= bk_cosh[k];
            sum += (k == 0) ? 0.5 * term : term;
            if (ex > 50.0 + t) break;
        }
        return sum * BK_H;
    }
    /* large x: the integrand is a narrow Gaussian-like bump; shrink h so
     * that exp(-2 pi^2/(h^2 x)) stays negligible. */
    double h = 0.5 / sqrt(x);
    double sum = 0.0;
    for (int k = 0; k < 100000; ++k) {
        double t = k * h;
        double sh = sinh(0.5 * t);
        double ex = 2.0 * x * sh * sh;
        double term = exp(-ex) * cosh(nu * t);
        if (kind) term /= cosh(t);
        sum += (k == 0) ? 0.5 * term : term;
        if (ex > 60.0) break;
    }
    return sum * h;
}

double or_bessel_k(double nu, double x)
{
    bk_init();
    return exp(-x) * bessel_scaled(nu, x, 0);
}

double or_bessel_ki(double nu, double x)
{
    bk_init();
    return exp(-x) * bessel_scaled(nu, x, 1);
}

/* ======================================================================== *
 * 3. Spectra.
 *
 * Eq. 2 with xi = chi_gamma/chi_e: y = xi/(3 chi_e (1-xi)), 2y = delta,
 * 3 chi_gamma y = xi^2/(1-xi), and d gamma_gamma = gamma_e d xi, so
 *   d^2N_gamma/dt dxi = alpha_f/(pi sqrt3 tau_c gamma_e) * B_gamma(xi),
 *   B_gamma = (2 + xi^2/(1-xi)) K_{2/3}(delta) - int_delta^inf K_{1/3}.
 * READING: the bracket printed in Eq. 2 has the opposite overall sign, which
 * is negative for every y > 0; we use the positive (standard) spectrum.
 *
 * Eq. 3 with eta = chi_-/chi_gamma.  READING: y is not redefined for Eq. 3;
 * we take y = chi_gamma/(3 chi_-(chi_gamma - chi_-)) = 1/(3 chi_gamma
 * eta (1-eta)), so 3 chi_gamma y = 1/(eta(1-eta)) and
 *   B_pm = int_delta^inf K_{1/3} + (1/(eta(1-eta)) - 2) K_{2/3}(delta),
 *   delta = 2/(3 chi_gamma eta (1-eta)).
 * ======================================================================== */
double or_emit_bracket(double chi_e, double xi)
{
    if (!(xi > 0.0) || !(xi < 1.0)) return 0.0;
    double delta = 2.0 * xi / (3.0 * chi_e * (1.0 - xi));
    return (2.0 + xi * xi / (1.0 - xi)) * or_bessel_k(2.0 / 3.0, delta)
           - or_bessel_ki(1.0 / 3.0, delta);
}

double or_pair_bracket(double chi_g, double eta)
{
    if (!(eta > 0.0) || !(eta < 1.0)) return 0.0;
    double e1 = eta * (1.0 - eta);
    double delta = 2.0 / (3.0 * chi_g * e1);
    return or_bessel_ki(1.0 / 3.0, delta) + (1.0 / e1 - 2.0) * or_bessel_k(2.0 / 3.0, delta);
}

/*
 * Quadrature variable.  Both spectra are integrated over s = logit of the
 * fraction (xi = 1/(1+e^-s), or eta likewise), which maps (0,1) to the real
 * line, turns the xi^(-2/3) endpoint behaviour into an exponential tail e^{s/3}
 * and keeps the integrand analytic; composite 20-point Gauss-Legendre panels
 * then give close to machine accuracy for totals and partial integrals alike.
 *
 * emit_f(s)  = B_gamma(xi(s)) dxi/ds
 * pair_f(s)  = B_pm(eta(s)) deta/ds * exp(8/(3 chi))   (scaled: the pair
 *              rate carries exp(-8/(3chi)) which would underflow at small chi)
 */
static double emit_f(double chi, double s)
{
    double es = exp(s);
    double xi = es / (1.0 + es);
    double omx = 1.0 / (1.0 + es);
    if (isinf(es)) { xi = 1.0; omx = 0.0; }
    double delta = 2.0 * es / (3.0 * chi);
    if (delta > 740.0) return 0.0;
    double k23 = bessel_scaled(2.0 / 3.0, delta, 0);
    double ki13 = bessel_scaled(1.0 / 3.0, delta, 1);
    double br = (2.0 + xi * es) * k23 - ki13;          /* e^delta B_gamma */
    return exp(-delta) * br * (xi * omx);
}

static double pair_f(double chi, double s)
{
    double c2 = cosh(0.5 * s), s2 = sinh(0.5 * s);
    double inv_e1 = 4.0 * c2 * c2;                       /* 1/(eta(1-eta)) */
    double delta = (8.0 / (3.0 * chi)) * c2 * c2;
    double excess = (8.0 / (3.0 * chi)) * s2 * s2;       /* delta - 8/(3chi) */
    if (excess > 740.0) return 0.0;
    double k23 = bessel_scaled(2.0 / 3.0, delta, 0);
    double ki13 = bessel_scaled(1.0 / 3.0, delta, 1);
    double br = ki13 + (inv_e1 - 2.0) * k23;             /* e^delta B_pm */
    return exp(-excess) * br / inv_e1;
}

/* 20-point Gauss-Legendre rule on [-1,1], nodes by Newton on P_20. */
#define GL_N 20
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GL_N; ++i) {
        double x = cos(M_PI * (i + 0.75) / (GL_N + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= GL_N; ++n) {
                double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1; p1 = p2;
            }
            dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        {
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= GL_N; ++n) {
                double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1; p1 = p2;
            }
            dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

typedef double (*spec_fn)(double chi, double s);

/* int_a^b f(chi, s) ds, optionally weighted by xi(s) (moment = 1) */
static double gl_panel(spec_fn f, double chi, double a, double b, int moment)
{
    double half = 0.5 * (b - a), mid = 0.5 * (b + a), sum = 0.0;
    for (int i = 0; i < GL_N; ++i) {
        double s = mid + half * gl_x[i];
        double v = f(chi, s);
        if (moment) v *= 1.0 / (1.0 + exp(-s));
        sum += gl_w[i] * v;
    }
    return sum * half;
}

/* panel layout over s for each spectrum */
typedef struct {
    int n;
    double edge[1200];
} panels;

static void emit_panels(double chi, panels *p)
{
    /* below s = -20 the integrand is a smooth e^{s/3} tail; above, the
     * double-exponential cut-off exp(-(2/(3chi)) e^s) needs finer panels. */
    double s_lo = -120.0, s_mid = -20.0;
    double s_hi = log(1.5 * chi * 760.0) + 0.5;
    int n = 0;
    for (double s = s_lo; s < s_mid - 1e-9; s += 2.0) p->edge[n++] = s;
    int nfine = (int)ceil((s_hi - s_mid) / 0.5);
    for (int k = 0; k <= nfine; ++k) p->edge[n++] = s_mid + (s_hi - s_mid) * k / nfine;
    p->n = n - 1;
}

static void pair_panels(double chi, panels *p)
{
    double S = acosh(1.0 + 570.0 * chi) + 0.25;
    int np = (int)ceil(2.0 * S / 0.25);
    if (np < 8) np = 8;
    for (int k = 0; k <= np; ++k) p->edge[k] = -S + 2.0 * S * k / np;
    p->n = np;
}

/* Mass of the emission integrand below the first panel edge s0.  For s -> -inf,
 * xi ~ e^s and K_{2/3}(delta) ~ (Gamma(2/3)/2)(2/delta)^{2/3}, so
 * emit_f(s) = C e^{s/3} (1 + O(e^{2s/3})) and the tail equals 3 emit_f(s0) up
 * to a relative O(e^{2 s0/3}).  The pair integrand has no such tail. */
static double lower_tail(spec_fn f, double chi, double s0)
{
    return (f == emit_f) ? 3.0 * emit_f(chi, s0) : 0.0;
}

static double spec_total(spec_fn f, double chi, const panels *p, int moment)
{
    double sum = moment ? 0.0 : lower_tail(f, chi, p->edge[0]);
    for (int k = 0; k < p->n; ++k) sum += gl_panel(f, chi, p->edge[k], p->edge[k + 1], moment);
    return sum;
}

double or_h_rad(double chi_e)
{
    gl_init(); bk_init();
    panels p; emit_panels(chi_e, &p);
    return spec_total(emit_f, chi_e, &p, 0) / (M_PI * sqrt(3.0));
}

/* Eq. 5: P_rad = int (d^2N/dt dgamma) gamma m c^2 dgamma.  READING: the
 * printed lower limit 1 is taken as 0, so that P_rad/P_cl depends on chi only:
 *   g = (sqrt3/(2 pi chi^2)) int_0^1 xi B_gamma dxi.                       */
double or_g(double chi_e)
{
    gl_init(); bk_init();
    panels p; emit_panels(chi_e, &p);
    return sqrt(3.0) / (2.0 * M_PI * chi_e * chi_e) * spec_total(emit_f, chi_e, &p, 1);
}

double or_h_pair(double chi_g)
{
    gl_init(); bk_init();
    panels p; pair_panels(chi_g, &p);
    return exp(-8.0 / (3.0 * chi_g)) * spec_total(pair_f, chi_g, &p, 0) / (M_PI * sqrt(3.0));
}

static double cdf_generic(spec_fn f, double chi, const panels *p, double s_target)
{
    double num = lower_tail(f, chi, p->edge[0]), tot = num;
    for (int k = 0; k < p->n; ++k) {
        double a = p->edge[k], b = p->edge[k + 1];
        double full = gl_panel(f, chi, a, b, 0);
        tot += full;
        if (b <= s_target) num += full;
        else if (a < s_target) num += gl_panel(f, chi, a, s_target, 0);
    }
    return num / tot;
}

double or_emit_cdf(double chi_e, double xi)
{
    gl_init(); bk_init();
    if (!(xi > 0.0)) return 0.0;
    if (!(xi < 1.0)) return 1.0;
    panels p; emit_panels(chi_e, &p);
    return cdf_generic(emit_f, chi_e, &p, log(xi) - log1p(-xi));
}

double or_pair_cdf(double chi_g, double eta)
{
    gl_init(); bk_init();
    if (!(eta > 0.0)) return 0.0;
    if (!(eta < 1.0)) return 1.0;
    panels p; pair_panels(chi_g, &p);
    return cdf_generic(pair_f, chi_g, &p, log(eta) - log1p(-eta));
}

/* ======================================================================== *
 * 4. Tables: rates at log-spaced chi nodes and quantiles of the CDF of
 *    Eq. 7 (emission) and of the pair CDF, at logit-spaced levels.
 *    READING: node layout, quantile levels and interpolation are not given
 *    by the paper; 128 log-spaced chi nodes and 128 logit levels in [-18,18].
 * ======================================================================== */

/* Solve CDF(s) = level for s, the CDF being the running integral over the
 * panels.  Levels below one half are solved on the lower running sum,
 * levels above on the upper (tail) sum so that the extreme quantiles keep
 * their relative accuracy.  Safeguarded Newton inside the bracketing panel. */
static double invert_level(spec_fn f, double chi, const panels *p,
                           const double *panel_int, const double *cum_lo,
                           const double *cum_hi, double total, double t_level)
{
    int upper = t_level > 0.0;
    /* r = 1/(1+e^-t) below one half; 1-r = 1/(1+e^t) above */
    double target = upper ? total / (1.0 + exp(t_level)) : total / (1.0 + exp(-t_level));
    int np = p->n, k;
    if (!upper) {
        for (k = 0; k < np - 1; ++k) if (cum_lo[k + 1] > target) break;
    } else {
        for (k = np - 1; k > 0; --k) if (cum_hi[k] > target) break;
    }
    double a = p->edge[k], b = p->edge[k + 1];
    double lo = a, hi = b;
    /* linear first guess inside the panel */
    double s = upper ? b - (target - cum_hi[k + 1]) / panel_int[k] * (b - a)
                     : a + (target - cum_lo[k]) / panel_int[k] * (b - a);
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double F, dF;
        if (!upper) { F = cum_lo[k] + gl_panel(f, chi, a, s, 0) - target; dF = f(chi, s); }
        else        { F = cum_hi[k + 1] + gl_panel(f, chi, s, b, 0) - target; dF = -f(chi, s); }
        /* F is increasing in s for the lower sum and decreasing for the tail */
        if ((F > 0.0) == (!upper)) hi = s; else lo = s;
        double sn = (dF != 0.0) ? s - F / dF : 0.5 * (lo + hi);
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) <= 1e-15 * (1.0 + fabs(s))) { s = sn; break; }
        s = sn;
        if (hi - lo <= 1e-15 * (1.0 + fabs(s))) break;
    }
    return s;
}

static void quantile_row(spec_fn f, double chi, const panels *p, int n_q,
                         double logit_max, double *row_s)
{
    double *pi = (double *)malloc(sizeof(double) * p->n);
    double *lo = (double *)malloc(sizeof(double) * (p->n + 1));
    double *hi = (double *)malloc(sizeof(double) * (p->n + 1));
    for (int k = 0; k < p->n; ++k) pi[k] = gl_panel(f, chi, p->edge[k], p->edge[k + 1], 0);
    lo[0] = lower_tail(f, chi, p->edge[0]);
    for (int k = 0; k < p->n; ++k) lo[k + 1] = lo[k] + pi[k];
    hi[p->n] = 0.0;
    for (int k = p->n - 1; k >= 0; --k) hi[k] = hi[k + 1] + pi[k];
    hi[0] += lo[0];
    for (int q = 0; q < n_q; ++q) {
        double t = -logit_max + 2.0 * logit_max * q / (n_q - 1);
        double total = (t > 0.0) ? hi[0] : lo[p->n];
        row_s[q] = invert_level(f, chi, p, pi, lo, hi, total, t);
    }
    free(pi); free(lo); free(hi);
}

int or_tables_compute(const or_table_spec *emit, const or_table_spec *pair,
                      double *ln_hrad, double *ln_g, double *emit_q,
                      double *pair_lnh, double *pair_q, int n_threads)
{
    gl_init(); bk_init();
    if (emit->n_chi < 2 || emit->n_q < 2 || pair->n_chi < 2 || pair->n_q < 2) return 1;
    int ne = emit->n_chi, npc = pair->n_chi;
    double le0 = log(emit->chi_min), le1 = log(emit->chi_max);
    double lp0 = log(pair->chi_min), lp1 = log(pair->chi_max);
    (void)n_threads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
    for (int job = 0; job < ne + npc; ++job) {
        if (job < ne) {
            int i = job;
            double chi = exp(le0 + (le1 - le0) * i / (ne - 1));
            panels p; emit_panels(chi, &p);
            double tot = spec_total(emit_f, chi, &p, 0);
            double mom = spec_total(emit_f, chi, &p, 1);
            ln_hrad[i] = log(tot / (M_PI * sqrt(3.0)));
            ln_g[i] = log(sqrt(3.0) / (2.0 * M_PI * chi * chi) * mom);
            double *row = emit_q + (size_t)i * emit->n_q;
            quantile_row(emit_f, chi, &p, emit->n_q, emit->logit_max, row);
            for (int q = 0; q < emit->n_q; ++q) row[q] = -log1p(exp(-row[q]));  /* ln xi */
        } else {
            int i = job - ne;
            double chi = exp(lp0 + (lp1 - lp0) * i / (npc - 1));
            panels p; pair_panels(chi, &p);
            double tot = spec_total(pair_f, chi, &p, 0);
            pair_lnh[i] = log(tot / (M_PI * sqrt(3.0)));            /* + 8/(3chi) implied */
            quantile_row(pair_f, chi, &p, pair->n_q, pair->logit_max,
                         pair_q + (size_t)i * pair->n_q);
        }
    }
    return 0;
}

void or_tables_bind(or_tables *t, const or_table_spec *emit, const or_table_spec *pair,
                    const double *ln_hrad, const double *ln_g, const double *emit_q,
                    const double *pair_lnh, const double *pair_q)
{
    t->e_n_chi = emit->n_chi; t->e_n_q = emit->n_q;
    t->e_chi_min = emit->chi_min;
    t->e_lnchi0 = log(emit->chi_min);
    t->e_inv_dlnchi = (emit->n_chi - 1) / (log(emit->chi_max) - log(emit->chi_min));
    t->e_logit_max = emit->logit_max;
    t->e_inv_dt = (emit->n_q - 1) / (2.0 * emit->logit_max);
    t->ln_hrad = ln_hrad; t->ln_g = ln_g; t->emit_q = emit_q;
    t->p_n_chi = pair->n_chi; t->p_n_q = pair->n_q;
    t->p_chi_min = pair->chi_min;
    t->p_lnchi0 = log(pair->chi_min);
    t->p_inv_dlnchi = (pair->n_chi - 1) / (log(pair->chi_max) - log(pair->chi_min));
    t->p_logit_max = pair->logit_max;
    t->p_inv_dt = (pair->n_q - 1) / (2.0 * pair->logit_max);
    t->pair_lnh = pair_lnh; t->pair_q = pair_q;
    t->e_interp = emit->interp; t->p_interp = pair->interp;
    t->emit_m = NULL; t->pair_m = NULL;
}

void or_tables_bind_spline(or_tables *t, const double *emit_m, const double *pair_m)
{
    t->emit_m = emit_m; t->pair_m = pair_m;
}

/* Natural cubic spline through y[0], y[s], ..., y[(n-1)s] at unit spacing h:
 * second derivatives M with M_0 = M_{n-1} = 0 and, inside,
 *   M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2,
 * solved by forward elimination and back substitution (the tridiagonal
 * system is diagonally dominant).  cp holds n scratch values. */
static void natural_spline_m(const double *y, ptrdiff_t s, int n, double h,
                             double *m, ptrdiff_t ms, double *cp)
{
    m[0] = 0.0;
    m[(n - 1) * ms] = 0.0;
    if (n < 3) return;
    /* unknowns k = 1..n-2; row k: 1 M_{k-1} + 4 M_k + 1 M_{k+1} = d_k */
    double prev_c = 0.0, prev_d = 0.0;
    for (int k = 1; k <= n - 2; ++k) {
        double d = 6.0 * (y[(k + 1) * s] - 2.0 * y[k * s] + y[(k - 1) * s]) / (h * h);
        double den = 4.0 - (k > 1 ? prev_c : 0.0);
        double c = (k < n - 2) ? 1.0 / den : 0.0;
        double dd = (d - (k > 1 ? prev_d : 0.0)) / den;
        cp[k] = c;
        m[k * ms] = dd;
        prev_c = c; prev_d = dd;
    }
    for (int k = n - 3; k >= 1; --k) m[k * ms] -= cp[k] * m[(k + 1) * ms];
}

void or_quantile_spline(const double *q, int n_chi, int n_q, double h_c, double h_t, double *m)
{
    const size_t N = (size_t)n_chi * n_q;
    double *mtt = m, *mcc = m + N, *mcctt = m + 2 * N;
    int nmax = n_chi > n_q ? n_chi : n_q;
    double *cp = (double *)malloc(sizeof(double) * (size_t)nmax);
    for (int i = 0; i < n_chi; ++i)             /* along t, each row */
        natural_spline_m(q + (size_t)i * n_q, 1, n_q, h_t, mtt + (size_t)i * n_q, 1, cp);
    for (int j = 0; j < n_q; ++j)               /* along ln chi, each column */
        natural_spline_m(q + j, n_q, n_chi, h_c, mcc + j, n_q, cp);
    for (int i = 0; i < n_chi; ++i)             /* the columns' curvature, along t */
        natural_spline_m(mcc + (size_t)i * n_q, 1, n_q, h_t, mcctt + (size_t)i * n_q, 1, cp);
    free(cp);
}

/* Linear interpolation in (ln chi, ln h).  Above the last node the end
 * segment is extended (READING: the paper gives no table range) and the
 * lookup is reported through *out_of_range.  Below the first node the
 * emission lookups follow their small-chi laws instead (see or_lookup_h_rad
 * and or_lookup_g). */
static double lerp_rate(const double *tab, int n, double lnchi0, double inv_d,
                        double chi, int *oor)
{
    double u = (log(chi) - lnchi0) * inv_d;
    int i;
    if (u < 0.0) i = 0;
    else if (u >= (double)(n - 1)) { i = n - 2; if (oor) *oor = 1; }
    else i = (int)u;
    double w = u - (double)i;
    return tab[i] + w * (tab[i + 1] - tab[i]);
}

/* READING (below the table): as chi -> 0 the photon-number rate of Eq. 2
 * becomes the classical one, proportional to chi (h_rad -> 5 chi/(2 sqrt 3)).
 * Below the first node h_rad is taken proportional to chi and equal to the
 * node value there, so the lookup is continuous and keeps the classical law. */
double or_lookup_h_rad(const or_tables *t, double chi, int *oor)
{
    if (!(chi > 0.0)) return 0.0;
    if (chi < t->e_chi_min) return exp(t->ln_hrad[0]) * (chi / t->e_chi_min);
    return exp(lerp_rate(t->ln_hrad, t->e_n_chi, t->e_lnchi0, t->e_inv_dlnchi, chi, oor));
}

/* READING (below the table): Eq. 5 must give the classical Larmor power as
 * chi -> 0, i.e. g -> 1, with g = 1 - (55 sqrt 3/16) chi + O(chi^2).  Below
 * the first node ln g is taken proportional to chi and equal to the node
 * value there: ln g(chi) = ln g(chi_min) chi/chi_min, which tends to 0 with
 * the first-order slope of the expansion. */
double or_lookup_g(const or_tables *t, double chi)
{
    if (!(chi > 0.0)) return 1.0;
    if (chi < t->e_chi_min) return exp(t->ln_g[0] * (chi / t->e_chi_min));
    return exp(lerp_rate(t->ln_g, t->e_n_chi, t->e_lnchi0, t->e_inv_dlnchi, chi, NULL));
}

double or_lookup_h_pair(const or_tables *t, double chi, int *oor)
{
    if (!(chi >= t->p_chi_min)) return 0.0;
    double v = lerp_rate(t->pair_lnh, t->p_n_chi, t->p_lnchi0, t->p_inv_dlnchi, chi, oor);
    return exp(v - 8.0 / (3.0 * chi));
}

/* Bilinear in (ln chi, logit r), chi clamped to the node range. */
static double bilerp_quantile(const double *q, int n_chi, int n_q, double lnchi0,
                              double inv_d, double logit_max, double inv_dt,
                              double chi, double r)
{
    double u = (log(chi) - lnchi0) * inv_d;
    if (!(u > 0.0)) u = 0.0;
    if (u > (double)(n_chi - 1)) u = (double)(n_chi - 1);
    int i = (int)u;
    if (i > n_chi - 2) i = n_chi - 2;
    double w = u - (double)i;
    /* logit of r; r = 1 gives +inf and lands on the top clamp */
    double t = log(r) - log(1.0 - r);
    if (!(t > -logit_max)) t = -logit_max;
    if (t > logit_max) t = logit_max;
    double v = (t + logit_max) * inv_dt;
    int j = (int)v;
    if (j > n_q - 2) j = n_q - 2;
    double z = v - (double)j;
    const double *r0 = q + (size_t)i * n_q, *r1 = r0 + n_q;
    double a = r0[j] + z * (r0[j + 1] - r0[j]);
    double b = r1[j] + z * (r1[j + 1] - r1[j]);
    return a + w * (b - a);
}

/* One cubic segment of a natural spline at fraction z of a step h:
 * (1-z) f0 + z f1 + h^2/6 [((1-z)^3 - (1-z)) m0 + (z^3 - z) m1]. */
static double spline_seg(double f0, double f1, double m0, double m1, double z, double h)
{
    double a = 1.0 - z;
    return a * f0 + z * f1 + ((a * a * a - a) * m0 + (z * z * z - z) * m1) * h * h / 6.0;
}

/* The tensor-product natural cubic spline of q at (ln chi, logit r), with the
 * node cell, weights and clamps of bilerp_quantile: the spline along t of
 * rows i and i+1 (and of their curvature in ln chi), then the spline along
 * ln chi between the two rows. */
static double bicubic_quantile(const double *q, const double *m, int n_chi, int n_q,
                               double lnchi0, double inv_d, double logit_max,
                               double inv_dt, double chi, double r)
{
    double u = (log(chi) - lnchi0) * inv_d;
    if (!(u > 0.0)) u = 0.0;
    if (u > (double)(n_chi - 1)) u = (double)(n_chi - 1);
    int i = (int)u;
    if (i > n_chi - 2) i = n_chi - 2;
    double w = u - (double)i;
    double t = log(r) - log(1.0 - r);
    if (!(t > -logit_max)) t = -logit_max;
    if (t > logit_max) t = logit_max;
    double v = (t + logit_max) * inv_dt;
    int j = (int)v;
    if (j > n_q - 2) j = n_q - 2;
    double z = v - (double)j;
    const double h_t = 1.0 / inv_dt, h_c = 1.0 / inv_d;
    const size_t N = (size_t)n_chi * n_q, a0 = (size_t)i * n_q + j, a1 = a0 + n_q;
    const double *mtt = m, *mcc = m + N, *mcctt = m + 2 * N;
    double f_i = spline_seg(q[a0], q[a0 + 1], mtt[a0], mtt[a0 + 1], z, h_t);
    double f_i1 = spline_seg(q[a1], q[a1 + 1], mtt[a1], mtt[a1 + 1], z, h_t);
    double c_i = spline_seg(mcc[a0], mcc[a0 + 1], mcctt[a0], mcctt[a0 + 1], z, h_t);
    double c_i1 = spline_seg(mcc[a1], mcc[a1 + 1], mcctt[a1], mcctt[a1 + 1], z, h_t);
    return spline_seg(f_i, f_i1, c_i, c_i1, w, h_c);
}

double or_sample_xi(const or_tables *t, double chi, double r)
{
    double lnxi = t->e_interp
        ? bicubic_quantile(t->emit_q, t->emit_m, t->e_n_chi, t->e_n_q, t->e_lnchi0, t->e_inv_dlnchi,
                           t->e_logit_max, t->e_inv_dt, chi, r)
        : bilerp_quantile(t->emit_q, t->e_n_chi, t->e_n_q, t->e_lnchi0, t->e_inv_dlnchi,
                          t->e_logit_max, t->e_inv_dt, chi, r);
    double xi = exp(lnxi);
    return xi < 1.0 ? xi : 1.0;
}

double or_sample_eta(const or_tables *t, double chi, double r)
{
    double s = t->p_interp
        ? bicubic_quantile(t->pair_q, t->pair_m, t->p_n_chi, t->p_n_q, t->p_lnchi0, t->p_inv_dlnchi,
                           t->p_logit_max, t->p_inv_dt, chi, r)
        : bilerp_quantile(t->pair_q, t->p_n_chi, t->p_n_q, t->p_lnchi0, t->p_inv_dlnchi,
                          t->p_logit_max, t->p_inv_dt, chi, r);
    return 1.0 / (1.0 + exp(-s));
}

/* ======================================================================== *
 * 5. Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
 *    (c0,c1,c2,c3) -> (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0))
 *    with the key bumped by the Weyl constants between rounds.
 *    The uniform draws xi, xi', xi'' of Sec. 3 are ((b>>11)+1) 2^-53, in ]0,1].
 * ======================================================================== */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_u01(uint64_t bits)
{
    return (double)((bits >> 11) + 1ULL) * (1.0 / 9007199254740992.0);
}

static void draw(uint64_t seed, uint64_t uid, uint32_t n_ev, uint64_t purpose, uint64_t out[4])
{
    uint64_t ctr[4] = { uid, (uint64_t)n_ev, purpose, 0ULL };
    uint64_t key[2] = { seed, 0ULL };
    or_philox4x64_10(ctr, key, out);
}

/* Sec. 3: a new particle's final optical depth tau^f = -log xi. */
static double initial_tau(uint64_t seed, uint64_t uid)
{
    uint64_t o[4];
    draw(seed, uid, 0, OR_RNG_INIT, o);
    return -log(or_u01(o[0]));
}

void or_init_tau(or_species *s, uint64_t seed)
{
    for (int64_t i = 0; i < s->n; ++i) s->tau[i] = initial_tau(seed, s->uid[i]);
}

/* ======================================================================== *
 * 6. Fields at a particle.
 * ======================================================================== */

/* Yee staggering of Ex Ey Ez Bx By Bz, in cells along x, y, z. */
static const double yee_stag[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

/* quadratic (triangular-shaped-cloud) weights around the nearest node */
static void tsc_weights(double g, int64_t *i0, double w[3])
{
    double f = floor(g + 0.5);
    double d = g - f;
    *i0 = (int64_t)f;
    w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (0.5 + d) * (0.5 + d);
}

void or_field_at(const or_field *f, double t, double x, double y, double z,
                 double E[3], double B[3])
{
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    if (f->kind == OR_FIELD_UNIFORM) {
        for (int c = 0; c < 3; ++c) { E[c] = f->E[c]; B[c] = f->B[c]; }
    } else if (f->kind == OR_FIELD_PLANE_WAVE) {
        /* Linearly polarised plane wave along +x from the vector potential
         * a_y(phi) = a0 sin^2(pi phi/Phi) sin(phi), phi = t - x, Phi = 2 pi N:
         * E_y = -da_y/dt = -a_y', B_z = da_y/dx = -a_y'. */
        double phi = t - x;
        double Phi = 2.0 * M_PI * f->n_periods;
        if (phi > 0.0 && phi < Phi) {
            double arg = M_PI * phi / Phi;
            double se = sin(arg), ce = cos(arg);
            double sp = sin(phi), cp = cos(phi);
            double da = f->a0 * ((M_PI / Phi) * (2.0 * se * ce) * sp + se * se * cp);
            E[1] = -da;
            B[2] = -da;
        }
    } else if (f->kind == OR_FIELD_YEE || f->kind == OR_FIELD_YEE_SEPARABLE) {
        double out[6];
        for (int c = 0; c < 6; ++c) {
            int64_t i0, j0, k0;
            double wx[3], wy[3], wz[3];
            tsc_weights((x - f->x0) / f->dx - yee_stag[c][0], &i0, wx);
            tsc_weights((y - f->y0) / f->dy - yee_stag[c][1], &j0, wy);
            tsc_weights((z - f->z0) / f->dz - yee_stag[c][2], &k0, wz);
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) {
                int64_t i = i0 - 1 + a;
                if (i < 0 || i >= f->nx) continue;
                for (int b = 0; b < 3; ++b) {
                    int64_t j = j0 - 1 + b;
                    if (j < 0 || j >= f->ny) continue;
                    for (int cc = 0; cc < 3; ++cc) {
                        int64_t k = k0 - 1 + cc;
                        if (k < 0 || k >= f->nz) continue;
                        double v;
                        if (f->kind == OR_FIELD_YEE)
                            v = (double)f->grid[c][(i * f->ny + j) * f->nz + k];
                        else   /* the node value the separable fill would store */
                            v = (double)(float)((f->a0 * f->tperp6[c * f->ny * f->nz + j * f->nz + k])
                                                * f->tpar6[c * f->nx + i]);
                        acc += (wx[a] * wy[b]) * wz[cc] * v;
                    }
                }
            }
            out[c] = acc;
        }
        E[0] = out[0]; E[1] = out[1]; E[2] = out[2];
        B[0] = out[3]; B[1] = out[4]; B[2] = out[5];
    }
}

/* Separable laser pulse on the Yee grid: value = (float)((a0 * T_perp[j,k]) * T_par[i]),
 * per component; tperp6 is [6][ny*nz], tpar6 is [6][nx]. */
void or_yee_fill_separable(float *grid6, int64_t nx, int64_t ny, int64_t nz,
                           double a0, const double *tperp6, const double *tpar6)
{
    int64_t plane = ny * nz, ncell = nx * plane;
    for (int c = 0; c < 6; ++c)
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t jk = 0; jk < plane; ++jk)
                grid6[c * ncell + i * plane + jk] =
                    (float)((a0 * tperp6[c * plane + jk]) * tpar6[c * nx + i]);
}

/* ======================================================================== *
 * 7. Quantum parameters, Eq. 1, in covariant form (equal to the printed
 *    E_par/E_perp form):
 *      chi_e     = sqrt((gamma E + u x B)^2 - (u.E)^2) / E_s
 *      chi_gamma = sqrt((|k| E + k x B)^2 - (k.E)^2) / E_s
 *    READING: "c x B" in the printed chi_gamma is c k_hat x B.
 * ======================================================================== */
static double chi_generic(double es_hat, double g, const double p[3],
                          const double E[3], const double B[3])
{
    double fx = g * E[0] + (p[1] * B[2] - p[2] * B[1]);
    double fy = g * E[1] + (p[2] * B[0] - p[0] * B[2]);
    double fz = g * E[2] + (p[0] * B[1] - p[1] * B[0]);
    double pe = p[0] * E[0] + p[1] * E[1] + p[2] * E[2];
    double q = (fx * fx + fy * fy + fz * fz) - pe * pe;
    return (q > 0.0 ? sqrt(q) : 0.0) / es_hat;
}

double or_chi_lepton(const or_units *u, const double p[3], double gamma,
                     const double E[3], const double B[3])
{
    return chi_generic(u->Es_hat, gamma, p, E, B);
}

double or_chi_photon(const or_units *u, const double k[3],
                     const double E[3], const double B[3])
{
    double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    return chi_generic(u->Es_hat, kk, k, E, B);
}

/* ======================================================================== *
 * 8. Lepton step (Secs. 2-3).
 *
 * Order within a step (READING: the paper does not fix it): fields at x^n;
 * Lorentz push u^{n-1/2} -> u_L (Boris); chi_e from (u_L, E, B); then either
 * the Sokolov continuous scheme (Eqs. 4-5) or the optical-depth Monte Carlo
 * (Eqs. 6-8); then x^{n+1} = x^n + dt dx/dt.
 * ======================================================================== */
static int append_ok(or_species *s)
{
    return s && s->n < s->capacity;
}

int or_push_emit(const or_tables *tab, const or_units *un, double q,
                 or_species *L, const or_field *f,
                 or_species *Pp, or_species *Pr,
                 const or_step *st, uint64_t *uid_next,
                 double *tally, int64_t *count)
{
    const double dt = st->dt, Es = un->Es_hat, tau0 = un->tau0_hat;
    /* the rate prefactor of Eq. 6, times the test switch rate_scale (exactly
     * A when it is 1, the default) */
    const double A = un->A_hat * (st->rate_scale > 0.0 ? st->rate_scale : 1.0);
    const double A_sok = un->A_hat;
    int overflow = 0;
    for (int64_t i = 0; i < L->n; ++i) {
        double x[3] = { L->x[i], L->y[i], L->z[i] };
        double u[3] = { L->ux[i], L->uy[i], L->uz[i] };
        double E[3], B[3];
        or_field_at(f, st->t, x[0], x[1], x[2], E, B);

        double g_old = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));

        /* --- Lorentz force f_l, Boris rotation ------------------------- */
        double h = 0.5 * q * dt;
        double um[3] = { u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2] };
        double gm = sqrt(1.0 + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]));
        double tv[3] = { h * B[0] / gm, h * B[1] / gm, h * B[2] / gm };
        double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
        double sv[3] = { 2.0 * tv[0] / (1.0 + t2), 2.0 * tv[1] / (1.0 + t2), 2.0 * tv[2] / (1.0 + t2) };
        double up[3] = { um[0] + (um[1] * tv[2] - um[2] * tv[1]),
                         um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                         um[2] + (um[0] * tv[1] - um[1] * tv[0]) };
        double uq[3] = { um[0] + (up[1] * sv[2] - up[2] * sv[1]),
                         um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                         um[2] + (up[0] * sv[1] - up[1] * sv[0]) };
        double uL[3] = { uq[0] + h * E[0], uq[1] + h * E[1], uq[2] + h * E[2] };
        double gL = sqrt(1.0 + (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
        tally[OR_T_WORK] += L->w[i] * (gL - g_old);

        /* --- chi_e, Eq. 1 ------------------------------------------------- */
        double chi = chi_generic(Es, gL, uL, E, B);
        double unew[3] = { uL[0], uL[1], uL[2] };
        double dv[3] = { 0.0, 0.0, 0.0 };
        int rad = st->rad_model;
        if (!isfinite(chi) || !isfinite(gL)) { count[OR_C_NAN]++; rad = OR_RAD_NONE; }

        if (rad == OR_RAD_SOKOLOV || (rad == OR_RAD_HYBRID && chi < st->chi_switch)) {
            /* --- Sokolov scheme, Eq. 4 with P_rad of Eq. 5 ----------------
             * READING (units of Eq. 4): delta_v = tau_0 (f_l - v (v.f_l))
             * / (1 + tau_0 v.f_l) in normalised units, and the delta_v x B
             * force carries the particle's charge q. */
            count[OR_C_SOKOLOV]++;
            double v[3] = { uL[0] / gL, uL[1] / gL, uL[2] / gL };
            double fl[3] = { q * (E[0] + (v[1] * B[2] - v[2] * B[1])),
                             q * (E[1] + (v[2] * B[0] - v[0] * B[2])),
                             q * (E[2] + (v[0] * B[1] - v[1] * B[0])) };
            double vf = v[0] * fl[0] + v[1] * fl[1] + v[2] * fl[2];
            double gq = chi > 0.0 ? or_lookup_g(tab, chi) : 1.0;
            /* alternative reading: delta_v with the quantum-reduced tau_0 g(chi) */
            double tq = (st->variants & OR_VAR_SOKOLOV_G) ? tau0 * gq : tau0;
            double den = 1.0 + tq * vf;
            for (int c = 0; c < 3; ++c) dv[c] = tq * (fl[c] - v[c] * vf) / den;
            double P = (2.0 / 3.0) * A_sok * chi * chi * gq;
            double dvB[3] = { dv[1] * B[2] - dv[2] * B[1],
                              dv[2] * B[0] - dv[0] * B[2],
                              dv[0] * B[1] - dv[1] * B[0] };
            for (int c = 0; c < 3; ++c) unew[c] = uL[c] + dt * (q * dvB[c] - P * uL[c] / gL);
            tally[OR_T_ERAD] += L->w[i] * P * dt;
        } else if (rad == OR_RAD_MC || rad == OR_RAD_HYBRID) {
            /* --- optical-depth Monte Carlo, Eqs. 6-8 -----------------------
             * tau holds tau^f - tau (what is left before the next emission);
             * dtau/dt = W = A h_rad(chi)/gamma (Eq. 6).  READING: several
             * emissions may fall in one step; each is placed at the local
             * time where tau reaches tau^f, up to max_events per step. */
            count[OR_C_MC]++;
            double p = sqrt(uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]);
            double uh[3] = { 0.0, 0.0, 0.0 };
            if (p > 0.0) { uh[0] = uL[0] / p; uh[1] = uL[1] / p; uh[2] = uL[2] / p; }
            double gam = gL, c_e = chi;
            int oor = 0;
            double W = (p > 0.0) ? A * or_lookup_h_rad(tab, c_e, &oor) / gam : 0.0;
            if (oor) { count[OR_C_RANGE]++; oor = 0; }
            double tau = L->tau[i], t_left = dt;
            int k = 0, emitted = 0;
            for (;;) {
                if (!(W > 0.0) || tau > W * t_left) { tau -= W * t_left; break; }
                if (k == st->max_events) { tau -= W * t_left; count[OR_C_CAP]++; break; }
                t_left -= (tau > 0.0 ? tau : 0.0) / W;
                uint64_t o[4];
                draw(st->seed, L->uid[i], L->n_ev[i], OR_RNG_EMIT, o);
                double r1 = or_u01(o[0]), r2 = or_u01(o[1]);
                /* Eq. 7 inverted: chi_gamma = xi chi_e; gamma_gamma = xi gamma_e */
                double xi = or_sample_xi(tab, c_e, r1);
                double gg = xi * gam;
                double wgt = L->w[i];
                count[OR_C_EMIT]++;
                if (gg > st->gamma_photon_min) {
                    /* Sec. 3: photon along the electron velocity, born at x^n,
                     * stored at level n+1: x^n + dt k_hat. */
                    double chig = xi * c_e;
                    or_species *dst = NULL;
                    int which;
                    if (Pp && chig > st->chi_photon_push_min) { dst = Pp; which = 0; }
                    else if (Pr) { dst = Pr; which = 1; }
                    else which = 2;
                    if (which == 2) {
                        count[OR_C_DROP]++; tally[OR_T_EDROP] += wgt * gg;
                    } else {
                        uint64_t nid = (*uid_next)++;
                        if (append_ok(dst)) {
                            int64_t j = dst->n++;
                            dst->x[j] = x[0] + dt * uh[0];
                            dst->y[j] = x[1] + dt * uh[1];
                            dst->z[j] = x[2] + dt * uh[2];
                            dst->ux[j] = gg * uh[0];
                            dst->uy[j] = gg * uh[1];
                            dst->uz[j] = gg * uh[2];
                            dst->w[j] = wgt;
                            dst->chi[j] = chig;
                            dst->uid[j] = nid;
                            dst->n_ev[j] = 0;
                            dst->tau[j] = initial_tau(st->seed, nid);
                        } else {
                            overflow = 1; count[OR_C_OVERFLOW]++;
                        }
                        if (which == 0) { count[OR_C_PUSH]++; tally[OR_T_EPUSH] += wgt * gg; }
                        else            { count[OR_C_REC]++;  tally[OR_T_EREC]  += wgt * gg; }
                    }
                } else {
                    /* READING: below 2 m c^2 no super-photon is created, the
                     * electron still recoils and the energy is tallied. */
                    count[OR_C_SUB]++; tally[OR_T_ESUB] += wgt * gg;
                }
                /* Eq. 8: p_f = (p - eps_gamma/c) p_hat, clamped at zero */
                if (!st->no_recoil) {
                    p = p - gg;
                    if (p < 0.0) p = 0.0;
                    gam = sqrt(1.0 + p * p);
                    double pv[3] = { p * uh[0], p * uh[1], p * uh[2] };
                    c_e = chi_generic(Es, gam, pv, E, B);
                    W = (p > 0.0) ? A * or_lookup_h_rad(tab, c_e, &oor) / gam : 0.0;
                    if (oor) { count[OR_C_RANGE]++; oor = 0; }
                }
                tau = -log(r2);              /* new tau^f = -log xi */
                L->n_ev[i]++;
                ++k; emitted = 1;
            }
            L->tau[i] = tau;
            if (emitted) { unew[0] = p * uh[0]; unew[1] = p * uh[1]; unew[2] = p * uh[2]; }
        }

        /* --- position: dx/dt = v (+ delta_v for Sokolov, Eq. 4) ---------- */
        double gn = sqrt(1.0 + (unew[0] * unew[0] + unew[1] * unew[1] + unew[2] * unew[2]));
        L->x[i] = x[0] + dt * (unew[0] / gn + dv[0]);
        L->y[i] = x[1] + dt * (unew[1] / gn + dv[1]);
        L->z[i] = x[2] + dt * (unew[2] / gn + dv[2]);
        L->ux[i] = unew[0]; L->uy[i] = unew[1]; L->uz[i] = unew[2];
    }
    return overflow;
}

/* ======================================================================== *
 * 9. Photon step (Sec. 3, pair creation with Eq. 3).
 *    dtau_gamma/dt = A h_pair(chi_gamma)/gamma_gamma for gamma_gamma > 2.
 *    At the event the photon is deleted and an e- e+ pair is created at its
 *    position; chi_- from P_pm(0 -> chi_-) = xi'', chi_+ = chi_gamma - chi_-.
 *    READING: energies gamma_pm = 1 + (gamma_gamma - 2) chi_pm/chi_gamma
 *    (total energy conserved), momenta along k_hat; the pair is stored at
 *    level n+1 (x^n + dt v_pm) and inherits the photon weight.
 * ======================================================================== */
int or_pair_create(const or_tables *tab, const or_units *un,
                   or_species *P, int64_t n_limit, const or_field *f,
                   or_species *Em, or_species *Ep,
                   const or_step *st, uint64_t *uid_next,
                   double *tally, int64_t *count)
{
    const double dt = st->dt, A = un->A_hat * (st->rate_scale > 0.0 ? st->rate_scale : 1.0);
    int overflow = 0;
    int64_t keep = 0;
    int64_t n_step = n_limit < P->n ? n_limit : P->n;
    for (int64_t j = 0; j < n_step; ++j) {
        double x[3] = { P->x[j], P->y[j], P->z[j] };
        double k[3] = { P->ux[j], P->uy[j], P->uz[j] };
        double E[3], B[3];
        or_field_at(f, st->t, x[0], x[1], x[2], E, B);
        double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        double chig = chi_generic(un->Es_hat, kk, k, E, B);
        int oor = 0;
        double W = (kk > 2.0) ? A * or_lookup_h_pair(tab, chig, &oor) / kk : 0.0;
        if (oor) count[OR_C_RANGE]++;
        count[OR_C_PHSTEP]++;
        double tau = P->tau[j] - W * dt;
        double kh[3] = { k[0] / kk, k[1] / kk, k[2] / kk };
        if (W > 0.0 && tau <= 0.0) {
            uint64_t o[4];
            draw(st->seed, P->uid[j], P->n_ev[j], OR_RNG_PAIR, o);
            double eta = or_sample_eta(tab, chig, or_u01(o[0]));
            double chim = eta * chig;
            double chip = chig - chim;
            double gmn, gpl, pm, pp;
            if (st->variants & OR_VAR_PAIR_MOMENTUM) {
                /* alternative reading: the photon momentum is split exactly */
                pm = (chim / chig) * kk;
                pp = (chip / chig) * kk;
                gmn = sqrt(1.0 + pm * pm);
                gpl = sqrt(1.0 + pp * pp);
            } else {
                gmn = 1.0 + (kk - 2.0) * (chim / chig);
                gpl = 1.0 + (kk - 2.0) * (chip / chig);
                pm = sqrt(gmn * gmn - 1.0);
                pp = sqrt(gpl * gpl - 1.0);
            }
            double wgt = P->w[j];
            count[OR_C_PAIR]++;
            tally[OR_T_EPAIR] += wgt * kk;
            for (int side = 0; side < 2; ++side) {
                or_species *D = side == 0 ? Em : Ep;
                double pmag = side == 0 ? pm : pp, gmag = side == 0 ? gmn : gpl;
                uint64_t nid = (*uid_next)++;
                if (append_ok(D)) {
                    int64_t m = D->n++;
                    double ux = pmag * kh[0], uy = pmag * kh[1], uz = pmag * kh[2];
                    D->x[m] = x[0] + dt * (ux / gmag);
                    D->y[m] = x[1] + dt * (uy / gmag);
                    D->z[m] = x[2] + dt * (uz / gmag);
                    D->ux[m] = ux; D->uy[m] = uy; D->uz[m] = uz;
                    D->w[m] = wgt;
                    if (D->chi) D->chi[m] = side == 0 ? chim : chip;
                    D->uid[m] = nid;
                    D->n_ev[m] = 0;
                    D->tau[m] = initial_tau(st->seed, nid);
                } else {
                    overflow = 1; count[OR_C_OVERFLOW]++;
                }
            }
            continue;  /* photon deleted */
        }
        /* survivor: straight line at c, stable compaction in place */
        P->x[keep] = x[0] + dt * kh[0];
        P->y[keep] = x[1] + dt * kh[1];
        P->z[keep] = x[2] + dt * kh[2];
        P->ux[keep] = k[0]; P->uy[keep] = k[1]; P->uz[keep] = k[2];
        P->tau[keep] = tau;
        P->w[keep] = P->w[j];
        P->chi[keep] = P->chi[j];
        P->uid[keep] = P->uid[j];
        P->n_ev[keep] = P->n_ev[j];
        ++keep;
    }
    /* photons created during this step (beyond n_limit) are first pushed at
     * the next step; they keep their order behind the survivors */
    for (int64_t j = n_step; j < P->n; ++j, ++keep) {
        P->x[keep] = P->x[j]; P->y[keep] = P->y[j]; P->z[keep] = P->z[j];
        P->ux[keep] = P->ux[j]; P->uy[keep] = P->uy[j]; P->uz[keep] = P->uz[j];
        P->tau[keep] = P->tau[j]; P->w[keep] = P->w[j]; P->chi[keep] = P->chi[j];
        P->uid[keep] = P->uid[j]; P->n_ev[keep] = P->n_ev[j];
    }
    P->n = keep;
    return overflow;
}

/* ======================================================================== *
 * 9b. The same steps on several OpenMP threads, for timing the oracle on all
 *     host cores: contiguous chunks run the serial steps above into private
 *     append buffers with ids from zero, then are joined in index order.
 * ======================================================================== */
static or_species species_view(const or_species *s, int64_t lo, int64_t n)
{
    or_species v = *s;
    v.x = s->x + lo; v.y = s->y + lo; v.z = s->z + lo;
    v.ux = s->ux + lo; v.uy = s->uy + lo; v.uz = s->uz + lo;
    v.tau = s->tau + lo; v.w = s->w + lo; v.chi = s->chi ? s->chi + lo : NULL;
    v.uid = s->uid + lo; v.n_ev = s->n_ev + lo;
    v.n = n; v.capacity = n;
    return v;
}

static or_species species_alloc(int64_t cap)
{
    or_species s;
    memset(&s, 0, sizeof s);
    s.capacity = cap;
    double **f[] = { &s.x, &s.y, &s.z, &s.ux, &s.uy, &s.uz, &s.tau, &s.w, &s.chi };
    for (int k = 0; k < 9; ++k) *f[k] = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    s.uid = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1));
    s.n_ev = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1));
    return s;
}

static void species_release(or_species *s)
{
    free(s->x); free(s->y); free(s->z); free(s->ux); free(s->uy); free(s->uz);
    free(s->tau); free(s->w); free(s->chi); free(s->uid); free(s->n_ev);
}

/* Append entry j of a chunk's buffer with its final id (optical depth drawn
 * for that id, as a new particle gets it); 0 if the buffer is full. */
static int append_with_id(or_species *dst, const or_species *src, int64_t j, uint64_t id, uint64_t seed)
{
    if (!append_ok(dst)) return 0;
    int64_t m = dst->n++;
    dst->x[m] = src->x[j]; dst->y[m] = src->y[j]; dst->z[m] = src->z[j];
    dst->ux[m] = src->ux[j]; dst->uy[m] = src->uy[j]; dst->uz[m] = src->uz[j];
    dst->w[m] = src->w[j];
    if (dst->chi) dst->chi[m] = src->chi[j];
    dst->uid[m] = id;
    dst->n_ev[m] = src->n_ev[j];
    dst->tau[m] = initial_tau(seed, id);
    return 1;
}

/* Photons of the chunks' two buffers carry ids local to their chunk, in the
 * chunk's serial emission order over both buffers; merging the two buffers
 * by id restores that order, and the chunk's id base makes it global. */
static int join_appends(or_species *dst0, or_species *dst1, or_species *b0, or_species *b1,
                        uint64_t base, uint64_t seed, int64_t *count)
{
    int overflow = 0;
    int64_t i0 = 0, i1 = 0;
    while (i0 < b0->n || i1 < b1->n) {
        int take0 = i1 >= b1->n || (i0 < b0->n && b0->uid[i0] < b1->uid[i1]);
        or_species *dst = take0 ? dst0 : dst1;
        or_species *src = take0 ? b0 : b1;
        int64_t j = take0 ? i0++ : i1++;
        if (!append_with_id(dst, src, j, base + src->uid[j], seed)) { overflow = 1; count[OR_C_OVERFLOW]++; }
    }
    return overflow;
}

int or_push_emit_omp(const or_tables *tab, const or_units *un, double q,
                     or_species *L, const or_field *f, or_species *Pp, or_species *Pr,
                     const or_step *st, uint64_t *uid_next, double *tally, int64_t *count, int n_threads)
{
    int nt = n_threads > 0 ? n_threads : 1;
    int64_t n = L->n;
    or_species *bp = (or_species *)calloc((size_t)nt, sizeof(or_species));
    or_species *br = (or_species *)calloc((size_t)nt, sizeof(or_species));
    uint64_t *ids = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    double *tal = (double *)calloc((size_t)nt * OR_T_N, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)nt * OR_C_N, sizeof(int64_t));
#pragma omp parallel for schedule(static, 1) num_threads(nt)
    for (int c = 0; c < nt; ++c) {
        int64_t lo = n * c / nt, hi = n * (c + 1) / nt;
        or_species lv = species_view(L, lo, hi - lo);
        int64_t cap = (hi - lo) * (st->max_events > 0 ? st->max_events : 1);
        bp[c] = species_alloc(Pp ? cap : 0);
        br[c] = species_alloc(Pr ? cap : 0);
        ids[c] = 0;
        or_push_emit(tab, un, q, &lv, f, Pp ? &bp[c] : NULL, Pr ? &br[c] : NULL, st, &ids[c],
                     tal + (size_t)c * OR_T_N, cnt + (size_t)c * OR_C_N);
    }
    int overflow = 0;
    uint64_t base = *uid_next;
    for (int c = 0; c < nt; ++c) {
        overflow |= join_appends(Pp, Pr, &bp[c], &br[c], base, st->seed, count);
        base += ids[c];
        for (int k = 0; k < OR_T_N; ++k) tally[k] += tal[(size_t)c * OR_T_N + k];
        for (int k = 0; k < OR_C_N; ++k) count[k] += cnt[(size_t)c * OR_C_N + k];
        species_release(&bp[c]);
        species_release(&br[c]);
    }
    *uid_next = base;
    free(bp); free(br); free(ids); free(tal); free(cnt);
    return overflow;
}

static void move_entries(or_species *s, int64_t to, int64_t from, int64_t m)
{
    if (m <= 0 || to == from) return;
    memmove(s->x + to, s->x + from, sizeof(double) * (size_t)m);
    memmove(s->y + to, s->y + from, sizeof(double) * (size_t)m);
    memmove(s->z + to, s->z + from, sizeof(double) * (size_t)m);
    memmove(s->ux + to, s->ux + from, sizeof(double) * (size_t)m);
    memmove(s->uy + to, s->uy + from, sizeof(double) * (size_t)m);
    memmove(s->uz + to, s->uz + from, sizeof(double) * (size_t)m);
    memmove(s->tau + to, s->tau + from, sizeof(double) * (size_t)m);
    memmove(s->w + to, s->w + from, sizeof(double) * (size_t)m);
    memmove(s->chi + to, s->chi + from, sizeof(double) * (size_t)m);
    memmove(s->uid + to, s->uid + from, sizeof(uint64_t) * (size_t)m);
    memmove(s->n_ev + to, s->n_ev + from, sizeof(uint32_t) * (size_t)m);
}

int or_pair_create_omp(const or_tables *tab, const or_units *un, or_species *P, int64_t n_limit,
                       const or_field *f, or_species *Em, or_species *Ep, const or_step *st,
                       uint64_t *uid_next, double *tally, int64_t *count, int n_threads)
{
    int nt = n_threads > 0 ? n_threads : 1;
    int64_t n_step = n_limit < P->n ? n_limit : P->n, tail = P->n - n_step;
    or_species *be = (or_species *)calloc((size_t)nt, sizeof(or_species));
    or_species *bq = (or_species *)calloc((size_t)nt, sizeof(or_species));
    int64_t *keep = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    uint64_t *ids = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    double *tal = (double *)calloc((size_t)nt * OR_T_N, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)nt * OR_C_N, sizeof(int64_t));
#pragma omp parallel for schedule(static, 1) num_threads(nt)
    for (int c = 0; c < nt; ++c) {
        int64_t lo = n_step * c / nt, hi = n_step * (c + 1) / nt;
        or_species pv = species_view(P, lo, hi - lo);
        be[c] = species_alloc(hi - lo);
        bq[c] = species_alloc(hi - lo);
        ids[c] = 0;
        or_pair_create(tab, un, &pv, hi - lo, f, &be[c], &bq[c], st, &ids[c],
                       tal + (size_t)c * OR_T_N, cnt + (size_t)c * OR_C_N);
        keep[c] = pv.n;
    }
    int overflow = 0;
    uint64_t base = *uid_next;
    int64_t kept = 0;
    for (int c = 0; c < nt; ++c) {
        int64_t lo = n_step * c / nt;
        move_entries(P, kept, lo, keep[c]);           /* survivors, stably */
        kept += keep[c];
        /* pairs: e- then e+ of each decay, ids two per pair in photon order */
        for (int64_t j = 0; j < be[c].n; ++j) {
            for (int side = 0; side < 2; ++side) {
                or_species *D = side == 0 ? Em : Ep;
                or_species *S = side == 0 ? &be[c] : &bq[c];
                if (!append_with_id(D, S, j, base + S->uid[j], st->seed)) { overflow = 1; count[OR_C_OVERFLOW]++; }
            }
        }
        base += ids[c];
        for (int k = 0; k < OR_T_N; ++k) tally[k] += tal[(size_t)c * OR_T_N + k];
        for (int k = 0; k < OR_C_N; ++k) count[k] += cnt[(size_t)c * OR_C_N + k];
        species_release(&be[c]);
        species_release(&bq[c]);
    }
    move_entries(P, kept, n_step, tail);              /* photons created this step */
    P->n = kept + tail;
    *uid_next = base;
    free(be); free(bq); free(keep); free(ids); free(tal); free(cnt);
    return overflow;
}

/* ======================================================================== *
 * 10. Cell ordering of a species (a PIC code's particle sort): stable by the
 *     key (i ny + j) nz + k of the Yee cell holding the particle, with
 *     i = floor((x - x0) * (1/dx)) etc.; particles outside the grid last.
 * ======================================================================== */
typedef struct { uint64_t key; int64_t idx; } or_keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const or_keyidx *p = (const or_keyidx *)a, *q = (const or_keyidx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx ? 1 : 0);
}

void or_sort_by_cell(or_species *s, int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                     double x0, double y0, double z0)
{
    or_sort_by_cell_bands(s, nx, ny, nz, dx, dy, dz, x0, y0, z0, 1);
}

/* energy band of |u|: floor(log2 |u|^2 / 6) clamped to [0, bands), from the exponent of |u|^2 */
static uint64_t energy_band(double ux, double uy, double uz, int32_t bands)
{
    double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
    int e = 0;
    if (u2 > 0.0 && isfinite(u2)) frexp(u2, &e);
    int b = (e - 1) >= 0 ? (e - 1) / 6 : 0;
    return (uint64_t)(b < bands - 1 ? b : bands - 1);
}

void or_sort_by_cell_bands(or_species *s, int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                           double x0, double y0, double z0, int32_t bands)
{
    int64_t n = s->n;
    if (n < 2) return;
    double idx_ = 1.0 / dx, idy = 1.0 / dy, idz = 1.0 / dz;
    uint64_t ncell = (uint64_t)(nx * ny * nz);
    or_keyidx *ki = (or_keyidx *)malloc(sizeof(or_keyidx) * n);
    for (int64_t i = 0; i < n; ++i) {
        double gx = (s->x[i] - x0) * idx_, gy = (s->y[i] - y0) * idy, gz = (s->z[i] - z0) * idz;
        uint64_t key = ncell;
        if (gx >= 0.0 && gy >= 0.0 && gz >= 0.0) {
            double fi = floor(gx), fj = floor(gy), fk = floor(gz);
            if (fi < (double)nx && fj < (double)ny && fk < (double)nz)
                key = (uint64_t)((((int64_t)fi * ny) + (int64_t)fj) * nz + (int64_t)fk);
        }
        if (bands > 1) key = key * (uint64_t)bands + energy_band(s->ux[i], s->uy[i], s->uz[i], bands);
        ki[i].key = key;
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(or_keyidx), cmp_keyidx);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *arr[9] = { s->x, s->y, s->z, s->ux, s->uy, s->uz, s->tau, s->w, s->chi };
    for (int a = 0; a < 9; ++a) {
        if (!arr[a]) continue;
        for (int64_t j = 0; j < n; ++j) tmp[j] = arr[a][ki[j].idx];
        memcpy(arr[a], tmp, sizeof(double) * n);
    }
    uint64_t *tu = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (int64_t j = 0; j < n; ++j) tu[j] = s->uid[ki[j].idx];
    memcpy(s->uid, tu, sizeof(uint64_t) * n);
    uint32_t *te = (uint32_t *)malloc(sizeof(uint32_t) * n);
    for (int64_t j = 0; j < n; ++j) te[j] = s->n_ev[ki[j].idx];
    memcpy(s->n_ev, te, sizeof(uint32_t) * n);
    free(tmp); free(tu); free(te); free(ki);
}

/* ======================================================================== *
 * 11. Merging of super-particles (coalescence).
 *
 * The paper asks only that merging keep energy and momentum (end of Sec. 3).
 * The scheme written here is the two-particle merge of Vranic et al.
 * (Comput. Phys. Commun. 191, 65 (2015)), which keeps weight, momentum and
 * energy exactly, so also on average:
 *  - a particle is eligible if it is alive (tau finite), inside the box of
 *    cells, of positive finite weight and with |u|^2 inside the energy range;
 *  - eligible particles are grouped by (cell, energy bin, direction bin);
 *    energy bins split each octave of |u|^2 into sub_bins equal parts of the
 *    mantissa; direction bins cut each face of the cube around the origin
 *    into n_dir x n_dir squares of the face coordinates u_a/|u_d|, u_b/|u_d|,
 *    d the axis of the largest |u| component (ties to the lower axis),
 *    a = d+1, b = d+2 (mod 3);
 *  - a group of at least min_group members becomes two particles of weight
 *    W/2 at the weighted mean position, each with the energy per unit weight
 *    E/W (E = sum w gamma, or sum w |k|) and momenta of equal size |u_new|
 *    at angles +-theta around P = sum w u, cos theta = |P| / (W |u_new|),
 *    in the plane of P and P x e_{d+1}, chi the weighted mean;
 *  - groups below min_group and ineligible particles are kept unchanged.
 * Output order: groups by (cell, momentum bin), members of a kept group in
 * input order, then the ineligible particles in input order.  New particles
 * take ids uid_next + (output slot) and a fresh optical depth; *uid_next
 * advances by the output count.
 * ======================================================================== */
typedef struct { uint64_t cell, mbin; int64_t idx; } or_mkey;

static int cmp_mkey(const void *a, const void *b)
{
    const or_mkey *p = (const or_mkey *)a, *q = (const or_mkey *)b;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    if (p->mbin != q->mbin) return p->mbin < q->mbin ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx ? 1 : 0);
}

/* momentum bin of u, or -1 if |u|^2 is outside the energy range */
static int64_t merge_mbin(const or_merge_spec *m, double ux, double uy, double uz, int *face_axis)
{
    double u[3] = { ux, uy, uz };
    double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
    if (!(u2 > 0.0) || !isfinite(u2)) return -1;
    int ex;
    double man = frexp(u2, &ex);                    /* u2 = man 2^ex, man in [0.5, 1) */
    int64_t oct = (int64_t)ex - 1 - m->octave_min;  /* u2 in [2^(ex-1), 2^ex)          */
    if (oct < 0 || oct >= m->n_octaves) return -1;
    int64_t sub = (int64_t)floor((2.0 * man - 1.0) * (double)m->sub_bins);
    int d = 0;
    if (fabs(u[1]) > fabs(u[d])) d = 1;
    if (fabs(u[2]) > fabs(u[d])) d = 2;
    double ud = fabs(u[d]);
    int64_t ia = (int64_t)floor((u[(d + 1) % 3] / ud + 1.0) * (0.5 * m->n_dir));
    int64_t ib = (int64_t)floor((u[(d + 2) % 3] / ud + 1.0) * (0.5 * m->n_dir));
    if (ia > m->n_dir - 1) ia = m->n_dir - 1;
    if (ib > m->n_dir - 1) ib = m->n_dir - 1;
    if (ia < 0) ia = 0;
    if (ib < 0) ib = 0;
    int64_t face = 2 * d + (u[d] < 0.0 ? 1 : 0);
    *face_axis = d;
    int64_t nd2 = (int64_t)m->n_dir * m->n_dir;
    return ((oct * m->sub_bins + sub) * 6 + face) * nd2 + ia * m->n_dir + ib;
}

static void copy_particle(const or_species *s, int64_t i, or_species *d, int64_t j)
{
    d->x[j] = s->x[i]; d->y[j] = s->y[i]; d->z[j] = s->z[i];
    d->ux[j] = s->ux[i]; d->uy[j] = s->uy[i]; d->uz[j] = s->uz[i];
    d->tau[j] = s->tau[i]; d->w[j] = s->w[i]; d->chi[j] = s->chi[i];
    d->uid[j] = s->uid[i]; d->n_ev[j] = s->n_ev[i];
}

static double mag3(const double u[3]) { return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

/* the two particles replacing the members k[a..b) of one group, at dst[o], dst[o+1] */
static void merge_group(const or_merge_spec *m, const or_species *src, const or_mkey *k, int64_t a, int64_t b,
                        or_species *dst, int64_t o, uint64_t seed, uint64_t base)
{
    /* sums over the group; energies relative to the first member, so that a
     * group of identical particles gives back their momentum */
    const int64_t i0 = k[a].idx;
    const double u0[3] = { src->ux[i0], src->uy[i0], src->uz[i0] };
    const double m0 = mag3(u0);
    const double e0 = m->massive ? sqrt(1.0 + m0 * m0) : m0;
    double W = 0.0, P[3] = { 0.0, 0.0, 0.0 }, S = 0.0, X[3] = { 0.0, 0.0, 0.0 }, Ch = 0.0;
    for (int64_t j = a; j < b; ++j) {
        const int64_t i = k[j].idx;
        const double w = src->w[i], u[3] = { src->ux[i], src->uy[i], src->uz[i] };
        const double mi = mag3(u);
        const double ei = m->massive ? sqrt(1.0 + mi * mi) : mi;
        W += w;
        for (int c = 0; c < 3; ++c) P[c] += w * u[c];
        S += w * (ei - e0);
        X[0] += w * src->x[i]; X[1] += w * src->y[i]; X[2] += w * src->z[i];
        Ch += w * src->chi[i];
    }
    int d;
    merge_mbin(m, u0[0], u0[1], u0[2], &d);
    const double eps = e0 + S / W;                     /* energy per unit weight */
    /* |u_new|: eps for photons; for leptons sqrt(eps^2 - 1), evaluated as
     * m0 + (eps - e0)(eps + e0)/(|u_new| + m0) */
    double un = eps;
    if (m->massive) {
        const double ur = sqrt(fmax((eps - 1.0) * (eps + 1.0), 0.0));
        un = (ur + m0 > 0.0) ? m0 + (S / W) * (eps + e0) / (ur + m0) : 0.0;
    }
    const double pn = mag3(P);
    double ph[3] = { 0.0, 0.0, 0.0 };
    if (pn > 0.0) {
        for (int c = 0; c < 3; ++c) ph[c] = P[c] / pn;
    } else {
        ph[d] = 1.0;
    }
    /* cos theta = |P| / (W |u_new|).  The gap G = W |u_new| - |P| is summed
     * as sum w (|u_new| - |u|) + sum w |u| |u_hat - P_hat|^2 / 2 (the first
     * sum is zero for photons), which keeps small angles accurate:
     * 1 - cos theta = G / (W |u_new|). */
    double G = 0.0;
    for (int64_t j = a; j < b; ++j) {
        const int64_t i = k[j].idx;
        const double w = src->w[i], u[3] = { src->ux[i], src->uy[i], src->uz[i] };
        const double mi = mag3(u);
        if (m->massive) G += w * (un - mi);
        if (mi > 0.0) {
            const double q[3] = { u[0] / mi - ph[0], u[1] / mi - ph[1], u[2] / mi - ph[2] };
            G += w * mi * 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        }
    }
    double omc = (W * un > 0.0) ? G / (W * un) : 0.0;  /* 1 - cos theta */
    if (omc < 0.0) omc = 0.0;
    if (omc > 1.0) omc = 1.0;
    const double ct = 1.0 - omc;
    const double st = sqrt(omc * (1.0 + ct));
    /* n = ph x e_{d+1}, normalised */
    const int e = (d + 1) % 3;
    double ev[3] = { 0.0, 0.0, 0.0 };
    ev[e] = 1.0;
    double nv[3] = { ph[1] * ev[2] - ph[2] * ev[1], ph[2] * ev[0] - ph[0] * ev[2], ph[0] * ev[1] - ph[1] * ev[0] };
    const double nn = mag3(nv);
    for (int c = 0; c < 3; ++c) nv[c] /= nn;
    for (int side = 0; side < 2; ++side, ++o) {
        const double sg = side == 0 ? 1.0 : -1.0;
        dst->x[o] = X[0] / W; dst->y[o] = X[1] / W; dst->z[o] = X[2] / W;
        dst->ux[o] = un * (ct * ph[0] + sg * st * nv[0]);
        dst->uy[o] = un * (ct * ph[1] + sg * st * nv[1]);
        dst->uz[o] = un * (ct * ph[2] + sg * st * nv[2]);
        dst->w[o] = 0.5 * W;
        dst->chi[o] = Ch / W;
        dst->uid[o] = base + (uint64_t)o;
        dst->n_ev[o] = 0;
        dst->tau[o] = initial_tau(seed, dst->uid[o]);
    }
}

int64_t or_merge(const or_merge_spec *m, const or_species *src, or_species *dst, uint64_t seed, uint64_t *uid_next)
{
    const int64_t n = src->n;
    const uint64_t ncell = (uint64_t)(m->nx * m->ny * m->nz);
    const double idx_ = 1.0 / m->dx, idy = 1.0 / m->dy, idz = 1.0 / m->dz;
    or_mkey *k = (or_mkey *)malloc(sizeof(or_mkey) * (n > 0 ? n : 1));
    int64_t live = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (isinf(src->tau[i]) && src->tau[i] > 0.0) continue;           /* decayed photon: dropped */
        uint64_t cell = ncell, mbin = 0;
        const double gx = (src->x[i] - m->x0) * idx_, gy = (src->y[i] - m->y0) * idy, gz = (src->z[i] - m->z0) * idz;
        if (gx >= 0.0 && gy >= 0.0 && gz >= 0.0) {
            const double fi = floor(gx), fj = floor(gy), fk = floor(gz);
            if (fi < (double)m->nx && fj < (double)m->ny && fk < (double)m->nz)
                cell = (uint64_t)((((int64_t)fi * m->ny) + (int64_t)fj) * m->nz + (int64_t)fk);
        }
        int d;
        const int64_t mb = merge_mbin(m, src->ux[i], src->uy[i], src->uz[i], &d);
        if (cell == ncell || mb < 0 || !(src->w[i] > 0.0) || !isfinite(src->w[i]))
            cell = ncell;                                                  /* kept as it is */
        else
            mbin = (uint64_t)mb;
        k[live].cell = cell; k[live].mbin = mbin; k[live].idx = i;
        ++live;
    }
    qsort(k, (size_t)live, sizeof(or_mkey), cmp_mkey);
    /* output count first, so that a short destination is refused untouched */
    int64_t n_out = 0;
    for (int64_t a = 0; a < live;) {
        int64_t b = a + 1;
        if (k[a].cell != ncell)
            while (b < live && k[b].cell == k[a].cell && k[b].mbin == k[a].mbin) ++b;
        n_out += (b - a >= m->min_group) ? 2 : (b - a);
        a = b;
    }
    if (n_out > dst->capacity) { free(k); return -1; }
    const uint64_t base = *uid_next;
    int64_t o = 0;
    for (int64_t a = 0; a < live;) {
        int64_t b = a + 1;
        if (k[a].cell != ncell)
            while (b < live && k[b].cell == k[a].cell && k[b].mbin == k[a].mbin) ++b;
        if (b - a < m->min_group) {
            for (int64_t j = a; j < b; ++j) copy_particle(src, k[j].idx, dst, o++);
        } else {
            merge_group(m, src, k, a, b, dst, o, seed, base);
            o += 2;
        }
        a = b;
    }
    dst->n = o;
    *uid_next = base + (uint64_t)o;
    free(k);
    return o;
}

/* ======================================================================== *
 * 12. Field solver and current deposition (coupling the step to a PIC loop).
 *
 * The paper's PIC code advances Maxwell's equations on a grid and deposits
 * the particles' currents (Sec. 1, Sec. 3); it does not describe how.  The
 * textbook choices are written here:
 *  - Yee's staggered finite differences (Yee 1966) in normalised units
 *    (c = 1): dB/dt = -curl E, dE/dt = curl B - J, on the staggering of the
 *    field gather (Ex at (i+1/2, j, k), ..., Bz at (i+1/2, j+1/2, k)),
 *    periodic in every direction, FP32 like the grid.  One advance: B by
 *    dt/2, E by dt with J, B by dt/2, so E and B sit at whole steps for the
 *    push;
 *  - charge-conserving deposition with quadratic (TSC) shapes (Esirkepov,
 *    Comput. Phys. Commun. 135, 144 (2001)): the change of a particle's
 *    node charges over the step is split into W_x + W_y + W_z, and
 *    J_x(i+1/2) - J_x(i-1/2) = -Q dx/dt W_x(i), J_x = 0 left of the stencil.
 * Node charges of a particle of weight w and charge q: Q S_x S_y S_z with
 * Q = q w j_scale, S the TSC weights around the nearest node of
 * g = (x - x0) (1/dx).
 * ======================================================================== */

static inline int64_t wrap(int64_t i, int64_t n) { i %= n; return i < 0 ? i + n : i; }

/* one half (h = dt/2) update of B from E */
static void yee_b_half(float *g, int64_t nx, int64_t ny, int64_t nz, float cx, float cy, float cz)
{
    const int64_t N = nx * ny * nz;
    const float *Ex = g, *Ey = g + N, *Ez = g + 2 * N;
    float *Bx = g + 3 * N, *By = g + 4 * N, *Bz = g + 5 * N;
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t k = 0; k < nz; ++k) {
                const int64_t c = (i * ny + j) * nz + k;
                const int64_t ip = (wrap(i + 1, nx) * ny + j) * nz + k;
                const int64_t jp = (i * ny + wrap(j + 1, ny)) * nz + k;
                const int64_t kp = (i * ny + j) * nz + wrap(k + 1, nz);
                /* B -= h curl E */
                Bx[c] = fmaf(cz, Ey[kp] - Ey[c], fmaf(-cy, Ez[jp] - Ez[c], Bx[c]));
                By[c] = fmaf(cx, Ez[ip] - Ez[c], fmaf(-cz, Ex[kp] - Ex[c], By[c]));
                Bz[c] = fmaf(cy, Ex[jp] - Ex[c], fmaf(-cx, Ey[ip] - Ey[c], Bz[c]));
            }
}

/* full update of E from B and J */
static void yee_e_full(float *g, const float *J, int64_t nx, int64_t ny, int64_t nz, float cx, float cy, float cz,
                       float dt)
{
    const int64_t N = nx * ny * nz;
    float *Ex = g, *Ey = g + N, *Ez = g + 2 * N;
    const float *Bx = g + 3 * N, *By = g + 4 * N, *Bz = g + 5 * N;
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t k = 0; k < nz; ++k) {
                const int64_t c = (i * ny + j) * nz + k;
                const int64_t im = (wrap(i - 1, nx) * ny + j) * nz + k;
                const int64_t jm = (i * ny + wrap(j - 1, ny)) * nz + k;
                const int64_t km = (i * ny + j) * nz + wrap(k - 1, nz);
                const float jx = J ? J[c] : 0.0f, jy = J ? J[N + c] : 0.0f, jz = J ? J[2 * N + c] : 0.0f;
                /* E += dt curl B - dt J */
                Ex[c] = fmaf(cy, Bz[c] - Bz[jm], fmaf(-cz, By[c] - By[km], fmaf(-dt, jx, Ex[c])));
                Ey[c] = fmaf(cz, Bx[c] - Bx[km], fmaf(-cx, Bz[c] - Bz[im], fmaf(-dt, jy, Ey[c])));
                Ez[c] = fmaf(cx, By[c] - By[im], fmaf(-cy, Bx[c] - Bx[jm], fmaf(-dt, jz, Ez[c])));
            }
}

void or_yee_advance(float *grid6, const float *J3, int64_t nx, int64_t ny, int64_t nz, double dx, double dy,
                    double dz, double dt)
{
    const float hx = (float)(0.5 * dt / dx), hy = (float)(0.5 * dt / dy), hz = (float)(0.5 * dt / dz);
    const float fx = (float)(dt / dx), fy = (float)(dt / dy), fz = (float)(dt / dz);
    yee_b_half(grid6, nx, ny, nz, hx, hy, hz);
    yee_e_full(grid6, J3, nx, ny, nz, fx, fy, fz, (float)dt);
    yee_b_half(grid6, nx, ny, nz, hx, hy, hz);
}

/* TSC weights of grid coordinate g around its nearest node n */
static void tsc3(double g, int64_t *n, double s[3])
{
    const double fn = floor(g + 0.5);
    const double d = g - fn;
    *n = (int64_t)fn;
    s[0] = 0.5 * (0.5 - d) * (0.5 - d);
    s[1] = 0.75 - d * d;
    s[2] = 0.5 * (0.5 + d) * (0.5 + d);
}

void or_deposit_charge(const or_species *s, double q, double j_scale, int64_t nx, int64_t ny, int64_t nz,
                       double dx, double dy, double dz, double x0, double y0, double z0, double *rho)
{
    const double ix = 1.0 / dx, iy = 1.0 / dy, iz = 1.0 / dz;
    for (int64_t p = 0; p < s->n; ++p) {
        if (isinf(s->tau[p]) && s->tau[p] > 0.0) continue;
        int64_t n[3];
        double S[3][3];
        tsc3((s->x[p] - x0) * ix, &n[0], S[0]);
        tsc3((s->y[p] - y0) * iy, &n[1], S[1]);
        tsc3((s->z[p] - z0) * iz, &n[2], S[2]);
        const double Q = q * s->w[p] * j_scale;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    const int64_t i = wrap(n[0] - 1 + a, nx), j = wrap(n[1] - 1 + b, ny), k = wrap(n[2] - 1 + c, nz);
                    rho[(i * ny + j) * nz + k] += Q * S[0][a] * S[1][b] * S[2][c];
                }
    }
}

int64_t or_deposit_current(const or_species *s, const double *xo, const double *yo, const double *zo, int64_t first,
                           double q, double j_scale, double dt, int64_t nx, int64_t ny, int64_t nz, double dx,
                           double dy, double dz, double x0, double y0, double z0, double *J)
{
    const double ix = 1.0 / dx, iy = 1.0 / dy, iz = 1.0 / dz;
    const double d[3] = { dx, dy, dz };
    const int64_t nn[3] = { nx, ny, nz };
    const int64_t N = nx * ny * nz;
    int64_t skipped = 0;
    for (int64_t p = first; p < s->n; ++p) {
        const double xn[3] = { s->x[p], s->y[p], s->z[p] };
        double xb[3];
        if (xo) {
            xb[0] = xo[p - first]; xb[1] = yo[p - first]; xb[2] = zo[p - first];
        } else {                                        /* created this step: back along u/gamma */
            const double u[3] = { s->ux[p], s->uy[p], s->uz[p] };
            const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int c = 0; c < 3; ++c) xb[c] = xn[c] - dt * (u[c] * ig);
        }
        const double org[3] = { x0, y0, z0 }, inv[3] = { ix, iy, iz };
        double S0[3][5] = { { 0 } }, S1[3][5] = { { 0 } }, D[3][5];
        int64_t base[3];
        int ok = 1;
        for (int c = 0; c < 3; ++c) {
            int64_t n0, n1;
            double s0[3], s1[3];
            tsc3((xb[c] - org[c]) * inv[c], &n0, s0);
            tsc3((xn[c] - org[c]) * inv[c], &n1, s1);
            if (n1 - n0 > 1 || n0 - n1 > 1) { ok = 0; break; }
            base[c] = n0 - 2;
            for (int a = 0; a < 3; ++a) {
                S0[c][1 + a] = s0[a];
                S1[c][(int)(n1 - n0) + 1 + a] = s1[a];
            }
            for (int a = 0; a < 5; ++a) D[c][a] = S1[c][a] - S0[c][a];
        }
        if (!ok) { ++skipped; continue; }
        const double Q = q * s->w[p] * j_scale;
        /* J_x: prefix along x of -Q dx/dt W_x, W_x = D_x (S_y S_z + D_y S_z/2 + S_y D_z/2 + D_y D_z/3) */
        for (int comp = 0; comp < 3; ++comp) {
            const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
            const double f = -Q * d[comp] / dt;
            for (int b = 0; b < 5; ++b)
                for (int c = 0; c < 5; ++c) {
                    const double t = S0[a1][b] * S0[a2][c] + 0.5 * D[a1][b] * S0[a2][c] + 0.5 * S0[a1][b] * D[a2][c]
                                     + D[a1][b] * D[a2][c] / 3.0;
                    double acc = 0.0;
                    for (int a = 0; a < 4; ++a) {
                        acc += f * D[comp][a] * t;
                        int64_t idx[3];
                        idx[comp] = wrap(base[comp] + a, nn[comp]);
                        idx[a1] = wrap(base[a1] + b, nn[a1]);
                        idx[a2] = wrap(base[a2] + c, nn[a2]);
                        J[comp * N + (idx[0] * ny + idx[1]) * nz + idx[2]] += acc;
                    }
                }
        }
    }
    return skipped;
}
