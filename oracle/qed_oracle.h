/*
 * qed_oracle.h -- CPU oracle for the per-particle radiation-and-QED step of
 * Lobet et al., "Modeling of radiative and quantum electrodynamics effects in
 * PIC simulations of ultra-relativistic laser-plasma interaction"
 * (arXiv:1311.1107).
 *
 * TEST INFRASTRUCTURE. This is the slow, serial, FP64 statement of what the
 * step computes, used only by the test-suite, by the smoke check and by the
 * CPU-baseline leg of the benchmark. The product (the HIP library) never
 * links, loads or calls it, and it shares no code, header, constant or table
 * generator with the product.
 *
 * Units are the normalised PIC units of the paper's setting: time 1/omega_r,
 * length c/omega_r, momentum m_e c, fields m_e c omega_r / e (E) and
 * m_e omega_r / e (B), with omega_r = 2 pi c / lambda.
 */
#ifndef QED_ORACLE_H
#define QED_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- constants and normalisation (Sec. 2, Eq. 1 and the definitions after
 *      Eqs. 1, 2 and 4) ---------------------------------------------------- */
typedef struct {
    double lambda;     /* reference wavelength [m]                           */
    double omega_r;    /* 2 pi c / lambda [1/s]                              */
    double alpha_f;    /* fine-structure constant                            */
    double E_s;        /* Schwinger field m^2 c^3/(e hbar) [V/m]             */
    double B_s;        /* E_s / c [T]                                        */
    double tau_c;      /* hbar/(m c^2) [s]                                   */
    double tau_0;      /* 2 e^2/(12 pi eps0 m c^3) [s]                       */
    double Es_hat;     /* E_s in units of m c omega_r / e                    */
    double A_hat;      /* alpha_f/(tau_c omega_r): rate prefactor             */
    double tau0_hat;   /* tau_0 omega_r                                      */
    double B_ref;      /* m omega_r / e [T]: unit of B                        */
    double E_ref;      /* m c omega_r / e [V/m]: unit of E                    */
} or_units;

void or_units_init(double lambda_m, or_units *u);

/* ---- special functions (integrands of Eqs. 2-3) -------------------------- */
double or_bessel_k(double nu, double x);    /* K_nu(x)                       */
double or_bessel_ki(double nu, double x);   /* int_x^inf K_nu(s) ds           */

/* Bracket of Eq. 2 (sign as in the standard synchrotron spectrum) as a
 * function of the photon fraction xi = chi_gamma/chi_e, and bracket of Eq. 3
 * as a function of eta = chi_-/chi_gamma. */
double or_emit_bracket(double chi_e, double xi);
double or_pair_bracket(double chi_g, double eta);

/* Total rates and the radiated-power ratio:
 *   dN_gamma/dt = alpha_f/(tau_c gamma_e) h_rad(chi_e)       (Eq. 6)
 *   P_rad = (2/3) alpha_f m c^2 chi_e^2/tau_c * g(chi_e)       (Eq. 5)
 *   dN_pm/dt  = alpha_f/(tau_c gamma_g) h_pair(chi_g)          (Eq. 3)   */
double or_h_rad(double chi_e);
double or_g(double chi_e);
double or_h_pair(double chi_g);
/* CDFs of Eq. 7 (emission, in xi) and of the pair spectrum (in eta).     */
double or_emit_cdf(double chi_e, double xi);
double or_pair_cdf(double chi_g, double eta);

/* ---- tables --------------------------------------------------------------
 * Rates tabulated at n_chi log-spaced nodes; quantiles at n_q logit levels
 * t_k = -L + 2 L k/(n_q-1), i.e. CDF levels r_k = 1/(1+exp(-t_k)).
 *   ln_hrad[i]      = ln h_rad(chi_i)
 *   ln_g[i]         = ln g(chi_i)
 *   emit_q[i*n_q+k] = ln xi  with P_gamma(xi; chi_i) = r_k
 *   pair_lnh[i]     = ln h_pair(chi_i) + 8/(3 chi_i)
 *   pair_q[i*n_q+k] = logit eta with P_pm(eta; chi_i) = r_k               */
/* interp: 0 bilinear in (ln chi, logit r); 1 the tensor-product natural
 * cubic spline through the same nodes (READING: the paper gives neither). */
typedef struct {
    double chi_min, chi_max;
    int32_t n_chi, n_q;
    double logit_max;
    int32_t interp, reserved;
} or_table_spec;

int or_tables_compute(const or_table_spec *emit, const or_table_spec *pair,
                      double *ln_hrad, double *ln_g, double *emit_q,
                      double *pair_lnh, double *pair_q, int n_threads);

typedef struct {
    /* emission side */
    int32_t e_n_chi, e_n_q;
    double e_chi_min, e_lnchi0, e_inv_dlnchi, e_logit_max, e_inv_dt;
    const double *ln_hrad, *ln_g, *emit_q;
    /* pair side */
    int32_t p_n_chi, p_n_q;
    double p_chi_min, p_lnchi0, p_inv_dlnchi, p_logit_max, p_inv_dt;
    const double *pair_lnh, *pair_q;
    /* quantile interpolation (or_table_spec.interp) and, for the spline, the
     * second-derivative tables of or_quantile_spline */
    int32_t e_interp, p_interp;
    const double *emit_m, *pair_m;
} or_tables;

void or_tables_bind(or_tables *t, const or_table_spec *emit, const or_table_spec *pair,
                    const double *ln_hrad, const double *ln_g, const double *emit_q,
                    const double *pair_lnh, const double *pair_q);

/* Second derivatives of the natural cubic splines through a quantile table
 * q[i*n_q+j] (n_chi rows at spacing h_c in ln chi, n_q columns at spacing h_t
 * in logit r), into m[3*n_chi*n_q]: m[0..N) = d2q/dt2 along each row,
 * m[N..2N) = d2q/dc2 along each column, m[2N..3N) = d2/dt2 along each row of
 * the second block (N = n_chi*n_q). */
void or_quantile_spline(const double *q, int n_chi, int n_q, double h_c, double h_t, double *m);
/* Attach the second-derivative tables of both quantile tables (needed when
 * the specs given to or_tables_bind ask for the spline). */
void or_tables_bind_spline(or_tables *t, const double *emit_m, const double *pair_m);

/* table lookups as the step uses them */
double or_lookup_h_rad(const or_tables *t, double chi, int *out_of_range);
double or_lookup_g(const or_tables *t, double chi);
double or_lookup_h_pair(const or_tables *t, double chi, int *out_of_range);
double or_sample_xi(const or_tables *t, double chi, double r);
double or_sample_eta(const or_tables *t, double chi, double r);

/* ---- counter-based random numbers: Philox4x64-10 (Salmon et al., SC'11) -- */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_u01(uint64_t bits);                   /* ((b>>11)+1) 2^-53 in (0,1] */

enum { OR_RNG_EMIT = 1, OR_RNG_PAIR = 2, OR_RNG_INIT = 3 };

/* ---- particles, fields, step -------------------------------------------- */
typedef struct {
    int64_t n, capacity;
    double *x, *y, *z, *ux, *uy, *uz;   /* u = p/(m c); photons: k, |k| = gamma_g */
    double *tau;                        /* optical depth left: tau^f - tau      */
    double *w;                          /* super-particle weight                 */
    double *chi;                        /* photons: chi_gamma at creation        */
    uint64_t *uid;
    uint32_t *n_ev;                     /* events so far (Philox counter word)   */
} or_species;

enum { OR_FIELD_UNIFORM = 0, OR_FIELD_PLANE_WAVE = 1, OR_FIELD_YEE = 2, OR_FIELD_YEE_SEPARABLE = 3 };

typedef struct {
    int32_t kind;
    double E[3], B[3];                 /* uniform field                           */
    double a0, n_periods;              /* plane wave a_y = a0 sin^2(pi phi/Phi) sin phi, phi = t - x */
    const float *grid[6];              /* Yee: Ex Ey Ez Bx By Bz, [i][j][k], k fastest */
    const double *tperp6, *tpar6;      /* Yee separable: node value (float)((a0 tperp[c][j,k]) tpar[c][i]) */
    int64_t nx, ny, nz;
    double dx, dy, dz, x0, y0, z0;
} or_field;

enum { OR_RAD_NONE = 0, OR_RAD_SOKOLOV = 1, OR_RAD_MC = 2, OR_RAD_HYBRID = 3 };

typedef struct {
    double t, dt;
    uint64_t seed;
    int32_t rad_model;
    double chi_switch;          /* HYBRID: Sokolov below, Monte Carlo above   */
    double gamma_photon_min;    /* photons stored only above this energy      */
    double chi_photon_push_min; /* stored photons go to the pushed buffer above this chi */
    int32_t max_events;         /* emissions per particle and step            */
    int32_t no_recoil;          /* test switch: emit without recoil           */
    int32_t variants;           /* alternative readings, OR of OR_VAR_*       */
    double rate_scale;          /* test switch: emission and pair rates times
                                   this (0 = 1), to find event decisions that
                                   lie within a relative margin of the rate   */
} or_step;

/* Alternative readings: the Sokolov delta_v of Eq. 4 with tau_0 g(chi)
 * instead of tau_0; a pair that splits the photon momentum exactly,
 * u_pm = (chi_pm/chi_gamma) k, instead of the energy. */
enum { OR_VAR_SOKOLOV_G = 1, OR_VAR_PAIR_MOMENTUM = 2 };

/* tallies (FP64 energies in m c^2 times weight, and event counts) */
enum { OR_T_WORK = 0, OR_T_ERAD, OR_T_EPUSH, OR_T_EREC, OR_T_EDROP, OR_T_ESUB,
       OR_T_EPAIR, OR_T_N = 8 };
enum { OR_C_EMIT = 0, OR_C_PUSH, OR_C_REC, OR_C_DROP, OR_C_SUB, OR_C_CAP,
       OR_C_RANGE, OR_C_SOKOLOV, OR_C_MC, OR_C_PAIR, OR_C_PHSTEP, OR_C_NAN,
       OR_C_OVERFLOW, OR_C_N = 16 };

void or_field_at(const or_field *f, double t, double x, double y, double z,
                 double E[3], double B[3]);
void or_yee_fill_separable(float *grid6, int64_t nx, int64_t ny, int64_t nz,
                           double a0, const double *tperp6, const double *tpar6);

double or_chi_lepton(const or_units *u, const double p[3], double gamma,
                     const double E[3], const double B[3]);
double or_chi_photon(const or_units *u, const double k[3],
                     const double E[3], const double B[3]);

void or_init_tau(or_species *s, uint64_t seed);

/* One step of the leptons of charge q (-1 electron, +1 positron), Secs. 2-3.
 * Returns 0, or 1 if an append did not fit (the overflow count says how many). */
int or_push_emit(const or_tables *tab, const or_units *u, double q,
                 or_species *lep, const or_field *f,
                 or_species *ph_push, or_species *ph_rec,
                 const or_step *st, uint64_t *uid_next,
                 double *tally, int64_t *count);

/* One step of the pushed photons [0, n_limit): Breit-Wheeler decay into pairs
 * (Sec. 3), straight-line push of the survivors and stable removal of decayed
 * photons.  Photons from n_limit on were created in the current step and are
 * left as they are (moved down behind the survivors).
 * The paper fixes only chi_+ = chi_gamma - chi_-.  The split of the energy,
 * gamma_pm = 1 + (gamma_gamma - 2) chi_pm/chi_gamma along the photon direction,
 * is a reading: pinned by energy and chi conservation, its partition is
 * parity unpinned by the paper. */
int or_pair_create(const or_tables *tab, const or_units *u,
                   or_species *ph, int64_t n_limit, const or_field *f,
                   or_species *elec, or_species *posi,
                   const or_step *st, uint64_t *uid_next,
                   double *tally, int64_t *count);

/* The same two steps on n_threads OpenMP threads (for timing the oracle on
 * all host cores).  The particles are cut into contiguous chunks, one per
 * thread; each chunk runs or_push_emit / or_pair_create as written, into its
 * own append buffers with ids counted from zero; the chunks are then joined
 * in index order: ids offset by the ids of the chunks before, the new
 * particles' optical depths drawn for their final ids, appends cut at the
 * buffers' capacities, survivors moved down.  Particles, ids, event
 * counters and counts are identical to the serial step; energy tallies are
 * summed per chunk, so they agree to rounding. */
int or_push_emit_omp(const or_tables *tab, const or_units *u, double q,
                     or_species *lep, const or_field *f,
                     or_species *ph_push, or_species *ph_rec,
                     const or_step *st, uint64_t *uid_next,
                     double *tally, int64_t *count, int n_threads);
int or_pair_create_omp(const or_tables *tab, const or_units *u,
                       or_species *ph, int64_t n_limit, const or_field *f,
                       or_species *elec, or_species *posi,
                       const or_step *st, uint64_t *uid_next,
                       double *tally, int64_t *count, int n_threads);

/* Stable reorder by Yee cell (i ny + j) nz + k, i = floor((x - x0)*(1/dx)) etc.;
 * particles outside the grid last. */
void or_sort_by_cell(or_species *s, int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                     double x0, double y0, double z0);
/* The same with key = cell key * bands + energy band of |u|, the band
 * floor(log2 |u|^2 / 6) clamped to [0, bands) (edges at |u| = 8, 64, 512). */
void or_sort_by_cell_bands(or_species *s, int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                           double x0, double y0, double z0, int32_t bands);

/* Merging of super-particles (coalescence; the paper fixes only that energy
 * and momentum are kept).  Two-particle merge per group of (cell, energy bin,
 * direction bin), keeping weight, momentum and energy: see the definition in
 * qed_oracle.c.  Decayed photons are dropped.  Returns the output count, or
 * -1 (dst untouched) if it exceeds dst->capacity. */
typedef struct {
    double x0, y0, z0, dx, dy, dz;      /* cells of the box                    */
    int64_t nx, ny, nz;
    int32_t massive;                    /* 1: leptons (energy gamma), 0: photons (|k|) */
    int32_t octave_min, n_octaves;      /* |u|^2 in [2^octave_min, 2^(octave_min+n_octaves)) */
    int32_t sub_bins;                   /* bins per octave of |u|^2 (power of two) */
    int32_t n_dir;                      /* direction bins per face edge          */
    int32_t min_group;                  /* groups this large or larger are merged */
} or_merge_spec;

int64_t or_merge(const or_merge_spec *m, const or_species *src, or_species *dst, uint64_t seed,
                 uint64_t *uid_next);

/* Field solver and current deposition (see section 12 of qed_oracle.c).
 * Grids are [component][nx][ny][nz] (z fastest), periodic in every direction.
 * or_yee_advance: B by dt/2, E by dt (minus dt J), B by dt/2, in FP32.
 * or_deposit_current: Esirkepov TSC currents of particles [first, n) moving
 * from (xo, yo, zo)[p - first] (or, if xo is NULL, from x - dt u/gamma) to
 * their present position, added to J3 (FP64); returns the number skipped for
 * moving more than one cell in some direction.
 * or_deposit_charge: TSC node charges q w j_scale S_x S_y S_z added to rho. */
void or_yee_advance(float *grid6, const float *J3, int64_t nx, int64_t ny, int64_t nz, double dx, double dy,
                    double dz, double dt);
int64_t or_deposit_current(const or_species *s, const double *xo, const double *yo, const double *zo, int64_t first,
                           double q, double j_scale, double dt, int64_t nx, int64_t ny, int64_t nz, double dx,
                           double dy, double dz, double x0, double y0, double z0, double *J3);
void or_deposit_charge(const or_species *s, double q, double j_scale, int64_t nx, int64_t ny, int64_t nz,
                       double dx, double dy, double dz, double x0, double y0, double z0, double *rho);

#ifdef __cplusplus
}
#endif
#endif
