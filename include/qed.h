/*
 * qed.h -- C interface of libqed, an MI355X (gfx950) implementation of the
 * per-particle radiation and QED step of Lobet et al., "Modeling of radiative
 * and quantum electrodynamics effects in PIC simulations of ultra-relativistic
 * laser-plasma interaction" (arXiv:1311.1107).
 *
 * For every super-particle the step gathers E and B, computes the Lorentz
 * invariant chi (Eq. 1) and advances the particle either with the Sokolov
 * radiation-damped push (Eqs. 4-5) or with the optical-depth Monte Carlo
 * (Eqs. 6-8), which emits super-photons; super-photons decay into e- e+ pairs
 * by the same Monte Carlo over the pair spectrum (Eq. 3, Sec. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: time 1/omega_r, length c/omega_r, momentum m_e c, E in
 *    m_e c omega_r/e, B in m_e omega_r/e, with omega_r = 2 pi c/lambda.
 *  - Every call returns a qed_status: QED_OK (0) or a negative error code.
 *    qed_last_error() returns a message for the calling host thread.
 *    Nothing is thrown across this interface.
 *  - Pointers marked [device] are device memory of the current HIP device;
 *    [host] pointers are host memory.  The caller owns all particle, field
 *    and tally memory; the library owns only qed_tables and qed_workspace
 *    handles.  Struct arguments themselves are host memory and are copied at
 *    the call; they may be reused immediately.
 *  - `stream` is a hipStream_t (NULL = legacy default stream).  Work is
 *    enqueued asynchronously; particle counts live in device memory, so a
 *    sequence of calls needs no host synchronisation and can be captured in
 *    a HIP graph.  Errors detected on the device (append past capacity,
 *    non-finite momenta, chi beyond the tables) are sticky in the workspace
 *    and read with qed_sync_status().
 *  - Particles are structure-of-arrays.  Within a launch, appended particles
 *    keep the serial order of their parents (stable append), so results do
 *    not depend on the launch configuration.
 *  - Random numbers are Philox4x64-10 keyed by (seed, 0) with counter
 *    (uid, n_event, purpose, 0): event decisions are reproducible for a given
 *    seed whatever the launch configuration or particle order.
 */
#ifndef QED_H
#define QED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qed_status;
#define QED_OK            0
#define QED_ERR_ARG      (-1)   /* invalid argument, detected on the host     */
#define QED_ERR_HIP      (-2)   /* a HIP runtime call or launch failed          */
#define QED_ERR_CAPACITY (-3)   /* an append did not fit (device, sticky)       */
#define QED_ERR_RANGE    (-4)   /* non-finite state met on the device (sticky)  */
#define QED_ERR_NOMEM    (-5)   /* allocation failed                            */

const char *qed_last_error(void);

/* ------------------------------------------------------------------------ *
 * Units (Sec. 2 definitions of E_s, alpha_f, tau_c; tau_0 after Eq. 4).
 * Es_hat = E_s in units of m c omega_r/e, A_hat = alpha_f/(tau_c omega_r)
 * (the rate prefactor of Eqs. 2, 3 and 6), tau0_hat = tau_0 omega_r.
 * ------------------------------------------------------------------------ */
typedef struct {
    double lambda;     /* [m]                                              */
    double omega_r;    /* [1/s]                                            */
    double alpha_f;
    double Es_hat;
    double A_hat;
    double tau0_hat;
} qed_units;

/* CODATA 2018 constants for the reference wavelength lambda_m [m] > 0. */
qed_status qed_units_init(double lambda_m, qed_units *out /* [host] */);

/* ------------------------------------------------------------------------ *
 * Rate and quantile tables (Eqs. 2, 3, 5, 6, 7 and the pair CDF of Sec. 3).
 *
 * Emission tables at n_chi log-spaced chi_e in [chi_min, chi_max]:
 *   ln_hrad[i]  = ln h_rad(chi_i), dN_gamma/dt = alpha_f h_rad/(tau_c gamma)
 *   ln_g[i]     = ln g(chi_i), P_rad = (2/3) alpha_f m c^2 chi^2 g/tau_c
 *   emit_q[i][k]= ln xi at CDF level r_k of Eq. 7 (xi = chi_gamma/chi_e),
 *                 r_k = 1/(1+exp(-t_k)), t_k = -L + 2 L k/(n_q-1), L = logit_max
 * Pair tables at n_chi log-spaced chi_gamma:
 *   pair_lnh[i] = ln h_pair(chi_i) + 8/(3 chi_i),
 *                 dN_pm/dt = alpha_f h_pair/(tau_c gamma_gamma)
 *   pair_q[i][k]= logit eta at level r_k of the pair CDF (eta = chi_-/chi_gamma)
 * Arrays are row-major, FP64.  Limits: 2 <= n_chi <= 256, 2 <= n_q <= 256,
 * 0 < chi_min < chi_max, logit_max > 0.
 *
 * interp selects how a quantile table is read between its nodes (the paper
 * samples Eq. 7 and the pair spectrum by inverting their CDFs but fixes no
 * interpolation): QED_INTERP_LINEAR, bilinear in (ln chi, logit r); or
 * QED_INTERP_SPLINE, the tensor-product natural cubic spline through the same
 * nodes (zero second derivative at the table edges), whose curvature tables
 * the library derives when the tables are loaded.  At 128 x 128 nodes the
 * CDF error of a sampled xi or eta is about 1e-3 bilinear and below 1e-5
 * with the spline.  reserved must be 0.
 * ------------------------------------------------------------------------ */
enum { QED_INTERP_LINEAR = 0, QED_INTERP_SPLINE = 1 };

typedef struct {
    double chi_min, chi_max;
    int32_t n_chi, n_q;
    double logit_max;
    int32_t interp;           /* QED_INTERP_LINEAR or QED_INTERP_SPLINE (quantile tables) */
    int32_t reserved;
} qed_table_spec;

typedef struct qed_tables qed_tables;          /* immutable device-resident tables */

/* FP64 Bessel quadrature on the host (multithreaded) into host arrays sized
 * n_chi, n_chi, n_chi*n_q (emission) and n_chi, n_chi*n_q (pair). */
qed_status qed_tables_compute_host(const qed_table_spec *emit, const qed_table_spec *pair,
                                   double *ln_hrad, double *ln_g, double *emit_q,
                                   double *pair_lnh, double *pair_q);
/* qed_tables_compute_host followed by upload to the current device. */
qed_status qed_tables_build(const qed_table_spec *emit, const qed_table_spec *pair,
                            qed_tables **out);
/* Upload tables given as host arrays (same layout as above), e.g. a saved set. */
qed_status qed_tables_load(const qed_table_spec *emit, const qed_table_spec *pair,
                           const double *ln_hrad, const double *ln_g, const double *emit_q,
                           const double *pair_lnh, const double *pair_q, qed_tables **out);
/* Copy one table back to the host: which = 0 ln_hrad, 1 ln_g, 2 emit_q,
 * 3 pair_lnh, 4 pair_q; n must equal its element count. */
qed_status qed_tables_export(const qed_tables *t, int32_t which, double *host, size_t n);
void qed_tables_free(qed_tables *t);

/* ------------------------------------------------------------------------ *
 * Particles (super-particles of Sec. 3), structure of arrays.
 * prec selects the element type of x..uz, w and chi: QED_F64 (double) or
 * QED_F32 (float).  tau is always FP64 (optical depth left before the next
 * event, tau^f - tau of Eq. 6).  For photons u holds k with |k| = gamma_gamma
 * and chi the chi_gamma at creation; for leptons chi may be NULL.
 * A photon whose tau is +INFINITY has decayed; qed_compact() removes it.
 * ------------------------------------------------------------------------ */
enum { QED_F64 = 0, QED_F32 = 1 };

typedef struct {
    int32_t prec;
    int32_t reserved;
    void *x, *y, *z;          /* [device] positions                              */
    void *ux, *uy, *uz;       /* [device] u = p/(m c)                            */
    double *tau;              /* [device]                                        */
    void *w;                  /* [device] weight                                 */
    void *chi;                /* [device] or NULL (leptons)                      */
    uint64_t *uid;            /* [device] unique id (Philox counter word 0)      */
    uint32_t *n_event;        /* [device] events so far (Philox counter word 1)  */
    int64_t *d_count;         /* [device] number of live entries                 */
    int64_t capacity;         /* [host] allocated entries                        */
} qed_species;

/* Sec. 3: initial optical depth tau^f = -log xi for entries [0, *d_count). */
qed_status qed_init_optical_depth(qed_species *s, uint64_t seed, void *stream);

/* ------------------------------------------------------------------------ *
 * External fields at the particles.
 *  UNIFORM:    E, B constant (the constant-field test of Sec. 4).
 *  PLANE_WAVE: linearly polarised along y, moving along +x, from the vector
 *              potential a_y = a0 sin^2(pi phi/Phi) sin(phi), phi = t - x,
 *              Phi = 2 pi n_periods: E_y = B_z = -da_y/dphi.
 *  YEE:        FP32 grid of 6 components Ex Ey Ez Bx By Bz, each [nx][ny][nz]
 *              (z fastest) on Yee staggered positions, gathered with quadratic
 *              (TSC) weights; zero outside the grid.
 * ------------------------------------------------------------------------ */
enum { QED_FIELD_UNIFORM = 0, QED_FIELD_PLANE_WAVE = 1, QED_FIELD_YEE = 2 };

typedef struct {
    int32_t kind;
    int32_t reserved;
    double E[3], B[3];
    double a0, n_periods;
    const float *grid;        /* [device] 6*nx*ny*nz floats                     */
    int64_t nx, ny, nz;
    double dx, dy, dz, x0, y0, z0;
    const float *bound;       /* [device] or NULL: field bounds from qed_field_bound  */
    int64_t bound_block;      /* cells per block edge of that table                */
} qed_field;

/* Bounds of a Yee field for the photon step.  For each block of block^3
 * cells (b = (bi nby + bj) nbz + bk, nb* = ceil(n* / block)) writes
 * bound[2 b] and bound[2 b + 1]: sqrt of the sum over the E (then B)
 * components of the largest |component| over the nodes the gather of a
 * particle in the block can touch (the block's nodes and two more on every
 * side), scaled up by 1 + 2^-20.  A particle outside the grid belongs to the
 * block of its nearest cell.  With f->bound = bound and f->bound_block =
 * block, the photon step skips the field gather of a wave whose photons all
 * have |k| (|E|_b + |B|_b) / E_s (1.01) below the pair table's chi_min: the
 * quantum parameter of Eq. 1 is at most |k| (|E| + |B|) / E_s, so their pair
 * rate is exactly zero with or without the gather and the results do not
 * change.  The table describes the grid at the time of the call; recompute
 * it whenever the grid changes.  bound [device] holds 2 nbx nby nbz floats;
 * 1 <= block <= 64; QED_ERR_ARG for a non-Yee field or a bad block. */
qed_status qed_field_bound(const qed_field *f, int32_t block, float *bound, void *stream);

/* Separable pulse onto the Yee grid: grid[c][i][j][k] =
 * (float)((a0 * tperp[c][j*nz+k]) * tpar[c][i]), tperp [device] 6*ny*nz,
 * tpar [device] 6*nx FP64. */
qed_status qed_yee_fill_separable(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                                  const double *tperp, const double *tpar, void *stream);

/* ------------------------------------------------------------------------ *
 * Step parameters.
 *  rad_model: NONE (Lorentz force only), SOKOLOV (Eqs. 4-5 for everyone),
 *  MC (Eqs. 6-8 for everyone), HYBRID (Sokolov where chi_e < chi_switch,
 *  Monte Carlo elsewhere: the classical and quantum regimes of Sec. 2).
 *  Emitted photons with gamma_gamma <= gamma_photon_min are not created
 *  (energy tallied; the paper's 2 m c^2 threshold, Sec. 3).  Created photons
 *  go to the pushed buffer if chi_gamma > chi_photon_push_min and that buffer
 *  is given, else to the recorded buffer if given, else are tallied only.
 *  max_events (1..4) bounds the emissions per particle and step.
 *  If d_step is not NULL the time is t + (*d_step) * dt (graph replays).
 * ------------------------------------------------------------------------ */
enum { QED_RAD_NONE = 0, QED_RAD_SOKOLOV = 1, QED_RAD_MC = 2, QED_RAD_HYBRID = 3 };

typedef struct {
    double t, dt;
    uint64_t seed;
    int32_t rad_model;
    int32_t max_events;
    double chi_switch;
    double gamma_photon_min;
    double chi_photon_push_min;
    int32_t no_recoil;        /* test switch: emit without recoil (frozen chi) */
    int32_t variants;         /* 0, or an OR of the QED_VAR_* model variants    */
    const int64_t *d_step;    /* [device] or NULL                               */
} qed_step;

/* Model variants (alternative readings of the paper; 0 = the default readings).
 *  QED_VAR_SOKOLOV_G:      the Sokolov correction delta_v of Eq. 4 is computed
 *                          with tau_0 g(chi_e) instead of the classical tau_0,
 *                          the same quantum reduction Eq. 5 applies to P_rad.
 *  QED_VAR_PAIR_MOMENTUM:  a pair splits the photon momentum exactly,
 *                          u_pm = (chi_pm / chi_gamma) k, gamma_pm =
 *                          sqrt(1 + |u_pm|^2) (Sec. 3 fixes only chi_+ =
 *                          chi_gamma - chi_-); the default keeps the energy
 *                          exact instead, gamma_pm = 1 + (gamma_gamma - 2)
 *                          chi_pm / chi_gamma along k.
 * Bits outside these are rejected (QED_ERR_ARG). */
enum { QED_VAR_SOKOLOV_G = 1, QED_VAR_PAIR_MOMENTUM = 2 };

/* ------------------------------------------------------------------------ *
 * Tallies: FP64 energies (m c^2 x weight), accumulated per tile slot so that
 * the sums are reproducible, and integer event counts (one set; integer sums
 * do not depend on order).  qed_tally_reduce() adds the energy slots in
 * slot order.
 * energy: 0 field work on leptons, 1 Sokolov radiated, 2 photons pushed,
 *   3 photons recorded, 4 photons tallied only, 5 below gamma_photon_min,
 *   6 photons converted to pairs.
 * count: 0 emissions, 1 pushed, 2 recorded, 3 tallied only, 4 below
 *   threshold, 5 max_events cap hit, 6 chi above table, 7 Sokolov steps,
 *   8 Monte Carlo steps, 9 pairs, 10 photon steps, 11 non-finite, 12 lost
 *   to capacity, 13 photon steps that skipped the field gather (field
 *   bounds, see qed_field_bound).
 * ------------------------------------------------------------------------ */
#define QED_N_ENERGY 8
#define QED_N_COUNT 16
typedef struct {
    double *energy;           /* [device] n_slots * QED_N_ENERGY, zeroed by caller */
    int64_t *count;           /* [device] QED_N_COUNT, zeroed by caller              */
    int64_t n_slots;          /* [host] >= 1; reproducible sums need one slot per tile:
                                 ceil(n / block) for the lepton step, ceil(n / 64) for the
                                 photon step; with fewer, slots are added to atomically */
} qed_tally;

qed_status qed_tally_reduce(const qed_tally *t, double energy[QED_N_ENERGY] /* [host] */,
                            int64_t count[QED_N_COUNT] /* [host] */, void *stream);

/* ------------------------------------------------------------------------ *
 * Workspace: per-tile append counts and their prefixes, emission records
 * handed from the physics pass to the append pass, look-back words and
 * tickets of the scan and compaction kernels, and the sticky device status.
 * max_particles bounds the capacity of any species passed with it;
 * max_leptons bounds the capacity of the lepton species given to
 * qed_push_emit (event items and emission records take about 272 bytes per
 * lepton in FP64).  One
 * workspace per stream; calls sharing a workspace must not overlap in time.
 * ------------------------------------------------------------------------ */
typedef struct qed_workspace qed_workspace;

qed_status qed_workspace_create(int64_t max_particles, int64_t max_leptons, qed_workspace **out);
void qed_workspace_free(qed_workspace *ws);

typedef struct {
    int64_t flags;            /* bit 0 capacity, bit 1 non-finite, bit 2 tally slots */
    int64_t needed[4];        /* largest count requested: photons pushed, photons
                                 recorded, electrons, positrons                    */
    int64_t chi_above_table;  /* lookups above the table's chi range              */
} qed_status_report;

/* Synchronises `stream`, copies the sticky status out, returns QED_OK,
 * QED_ERR_CAPACITY or QED_ERR_RANGE accordingly and clears it if clear != 0. */
qed_status qed_sync_status(qed_workspace *ws, qed_status_report *out /* [host] */,
                           int32_t clear, void *stream);

/* Launch shape of the persistent kernels: threads per block (64, 128, 192
 * or 256), particles per thread (1), blocks per compute unit (1..64) and an
 * optional cap on the persistent grid (max_blocks >= 8, rounded down to a
 * multiple of 8; 0 = no cap).  The grid is min(CUs x blocks_per_cu, tiles of
 * the species' capacity, max_blocks), rounded to a multiple of 8; each block
 * then walks as many tiles as the live count needs, so a small cap makes
 * every block loop over many tiles.  Zero fields take the library defaults
 * (256, 1, 8, no cap).  Results do not depend on the schedule. */
typedef struct {
    int32_t block;
    int32_t items_per_thread;
    int32_t blocks_per_cu;
    int32_t max_blocks;
} qed_schedule;

/* ------------------------------------------------------------------------ *
 * One step of the leptons of `charge` (-1 electrons, +1 positrons), Secs. 2-3:
 * field at x^n, Lorentz push to u^{n+1/2}, chi_e (Eq. 1), Sokolov (Eqs. 4-5)
 * or optical-depth Monte Carlo emission (Eqs. 6-8) with photon appends, then
 * x^{n+1}.  New photons are stored at level n+1 (x^n + dt k_hat), with
 * k = gamma_gamma u_hat (collinear emission, Sec. 3) and ids from *d_uid_next.
 * ph_push / ph_rec may be NULL.  sched may be NULL.
 * ------------------------------------------------------------------------ */
qed_status qed_push_emit(const qed_tables *tab, qed_workspace *ws, const qed_units *u,
                         double charge, qed_species *lep, const qed_field *f,
                         qed_species *ph_push, qed_species *ph_rec, qed_tally *tally,
                         const qed_step *st, uint64_t *d_uid_next /* [device] */,
                         const qed_schedule *sched, void *stream);

/* The same step as qed_push_emit for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no qed_workspace; the look-back words, per-tile counts and emission
 * records live in a static device array of the library (about 18.0 MB,
 * held on each GPU the library runs on until the process ends), and the call
 * makes no allocation.  lep->capacity must not exceed 65536 (QED_ERR_ARG
 * otherwise).  d_status [device] is 6 words the caller zeroes once: the call
 * ORs its status flags into d_status[0] (bit 0 capacity, bit 1 non-finite)
 * and raises d_status[1..4] (needed counts: photons pushed, photons
 * recorded) and d_status[5] to the largest value seen, as qed_sync_status
 * reports them for a workspace.  Every call on one GPU shares the array:
 * calls must be ordered (one stream, or synchronised), since overlapping
 * calls on one GPU race.  The first call on a device sets the array up and
 * synchronises that device, so it must not be made under graph capture. */
qed_status qed_push_emit_static(const qed_tables *tab, const qed_units *u, double charge,
                                qed_species *lep, const qed_field *f, qed_species *ph_push,
                                qed_species *ph_rec, qed_tally *tally, const qed_step *st,
                                uint64_t *d_uid_next /* [device] */, uint64_t *d_status /* [device] */,
                                const qed_schedule *sched, void *stream);

/* One step of pushed photons (Sec. 3 with Eq. 3): chi_gamma, optical depth
 * against the pair rate, decay into an e- e+ pair at the photon's position
 * (chi_- from the pair CDF, chi_+ = chi_gamma - chi_-, energies
 * 1 + (gamma_gamma - 2) chi_pm/chi_gamma along k_hat), straight-line push of
 * the others.  Decayed photons get tau = +INFINITY (see qed_compact). */
qed_status qed_pair_create(const qed_tables *tab, qed_workspace *ws, const qed_units *u,
                           qed_species *ph, const qed_field *f, qed_species *elec,
                           qed_species *posi, qed_tally *tally, const qed_step *st,
                           uint64_t *d_uid_next /* [device] */, const qed_schedule *sched,
                           void *stream);

/* Stable in-place removal of decayed photons (tau == +INFINITY). */
qed_status qed_compact(qed_workspace *ws, qed_species *ph, const qed_schedule *sched,
                       void *stream);

/* ------------------------------------------------------------------------ *
 * Batched form: many independent bunches, concatenated in `lep`, each in its
 * own plane wave, advanced by one persistent launch.  offsets [device] has
 * n_bunches+1 entries (bunch b is [offsets[b], offsets[b+1])), a0 and
 * n_periods [device] one per bunch; *lep->d_count must equal offsets[n_bunches].
 * Appends follow bunch order, then particle order.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_bunches;
    int32_t reserved;
    const int64_t *offsets;   /* [device] */
    const double *a0;         /* [device] */
    const double *n_periods;  /* [device] */
} qed_bunches;

qed_status qed_push_emit_batched(const qed_tables *tab, qed_workspace *ws, const qed_units *u,
                                 double charge, qed_species *lep, const qed_bunches *b,
                                 qed_species *ph_push, qed_species *ph_rec, qed_tally *tally,
                                 const qed_step *st, uint64_t *d_uid_next,
                                 const qed_schedule *sched, void *stream);

/* Autotuner: times each candidate schedule of qed_push_emit_batched over
 * `trial_steps` steps on a scratch copy of the lepton state (the caller's
 * particles, counters and tallies are left as they were) and returns the
 * fastest in *best.  candidates [host] has n_candidates entries; if cache_path
 * is not NULL, a result stored there for the same problem is reused and a new
 * one is written (one text line per problem: its key, then block,
 * items_per_thread, blocks_per_cu, max_blocks and the time per step). */
qed_status qed_autotune_batched(const qed_tables *tab, qed_workspace *ws, const qed_units *u,
                                double charge, qed_species *lep, const qed_bunches *b,
                                qed_species *ph_rec, const qed_step *st,
                                const qed_schedule *candidates, int32_t n_candidates,
                                int32_t trial_steps, const char *cache_path,
                                qed_schedule *best, double *best_ms, void *stream);

/* ------------------------------------------------------------------------ *
 * Cell ordering.  Writes the particles of src into dst (same precision,
 * capacity >= src's) ordered by the Yee cell that holds them: key
 * (i ny + j) nz + k with i = floor((x - x0)/dx) etc., particles outside the
 * grid after all cells; equal keys keep their order (stable), so the result
 * is a deterministic function of src.  Decayed photons (tau = +INFINITY) are
 * dropped; *dst->d_count receives the number kept.  Keeps the field gather
 * of neighbouring threads on shared grid lines.  grid supplies the geometry
 * (kind QED_FIELD_YEE).  The sorter holds 16 bytes per particle of scratch
 * (device memory, owned by the caller until qed_sorter_free); max_particles
 * must be below 2^32 - 1.  src and dst are device species in distinct
 * buffers; the workspace lends its look-back scratch, so calls on one
 * workspace are ordered on one stream.  QED_ERR_ARG for a null argument,
 * a non-Yee geometry or more than 2^31 cells, differing precisions or chi
 * arrays, aliased buffers, dst->capacity < src->capacity, or
 * src->capacity above the sorter's maximum; QED_ERR_HIP if a launch fails.
 * ------------------------------------------------------------------------ */
typedef struct qed_sorter qed_sorter;
qed_status qed_sorter_create(int64_t max_particles, qed_sorter **out);
void qed_sorter_free(qed_sorter *s);
qed_status qed_sort_by_cell(qed_sorter *s, qed_workspace *ws, qed_species *src, qed_species *dst,
                            const qed_field *grid, void *stream);
/* The same order with each cell's particles grouped by energy band:
 * key = cell key * bands + b, b = min(bands - 1, floor(log2 |u|^2 / 6)) (0 for
 * |u| < 8), taken from the exponent of |u|^2 = fma(uz, uz, fma(uy, uy, ux ux))
 * in FP64: band edges at |u| = 8, 64, 512, ...  bands is 1 (qed_sort_by_cell),
 * 2, 4 or 8.  Photons of similar energy then share waves, which lets the
 * photon step skip whole waves' gathers (qed_field_bound). */
qed_status qed_sort_by_cell_bands(qed_sorter *s, qed_workspace *ws, qed_species *src, qed_species *dst,
                                  const qed_field *grid, int32_t bands, void *stream);

/* ------------------------------------------------------------------------ *
 * Log-binned energy spectrum of a species (the photon and lepton spectra the
 * paper's diagnostics compare, Sec. 4).  The energy of entry i is
 * e = |u| for photons (photons != 0: |k| = gamma_gamma) or e = sqrt(1+|u|^2)
 * (the Lorentz factor) for leptons, taken in FP64 for either precision.  Its
 * bin is b = 1 + floor(n_bins * ln(e/e_min) / ln(e_max/e_min)) for
 * e_min <= e < e_max, 0 below e_min (and for e = 0 or non-finite e), and
 * n_bins + 1 at or above e_max.  Entries [0, *d_count) are counted; decayed
 * photons (tau = +-INFINITY) are skipped.  The call ADDS to
 * count[n_bins + 2] [device] (entries per bin) and wsum[n_bins + 2]
 * [device] (the sum over the bin of round(w * weight_scale), in integers so
 * that the sums do not depend on the order of the additions; weights that
 * are multiples of 1/weight_scale are summed exactly).  1 <= n_bins <= 1024,
 * 0 < e_min < e_max, weight_scale > 0; QED_ERR_ARG otherwise.
 * ------------------------------------------------------------------------ */
qed_status qed_spectrum(const qed_species *s, int32_t photons, double e_min, double e_max, int32_t n_bins,
                        double weight_scale, int64_t *count, int64_t *wsum, void *stream);

/* ------------------------------------------------------------------------ *
 * Merging of super-particles (coalescence).  The paper requires only that a
 * merge keep energy and momentum (end of Sec. 3); this is the two-particle
 * merge of Vranic et al. (Comput. Phys. Commun. 191, 65 (2015)), which keeps
 * weight, momentum and energy exactly.
 *  Eligible: alive (tau not +INFINITY), inside the box of cells
 *  (i = floor((x - x0) * (1/dx)) in [0, nx) etc.), weight > 0 and finite,
 *  |u|^2 in [2^octave_min, 2^(octave_min + n_octaves)).
 *  Groups: eligible particles with equal (cell, energy bin, direction bin).
 *  With |u|^2 = m 2^e (frexp, m in [0.5, 1)) the energy bin is
 *  (e - 1 - octave_min) * sub_bins + floor((2m - 1) sub_bins).  The
 *  direction bin: face 2d + (u_d < 0), d the axis of the largest |u_c|
 *  (ties to the lower axis), then floor((u_c/|u_d| + 1) n_dir / 2) (clamped
 *  to n_dir - 1) for c = d+1 and d+2 (mod 3).  All in FP64 for either
 *  precision, |u|^2 as fma(uz, uz, fma(uy, uy, ux ux)).
 *  A group of at least min_group members becomes two particles: weight W/2
 *  each (W the group's weight), the weighted mean position and chi, energy
 *  per unit weight E/W (E = sum w gamma for leptons, sum w |k| for photons),
 *  momenta of equal size |u_new| at angles +-theta about P = sum w u with
 *  cos theta = |P| / (W |u_new|), split along P x e_(d+1); new ids
 *  *d_uid_next + (output index), n_event 0, tau drawn as in
 *  qed_init_optical_depth with seed.  Smaller groups and ineligible
 *  particles are copied unchanged; decayed photons are dropped.
 *  Order of dst: groups by (cell, bin) ascending, members of a copied group
 *  in src order; then the ineligible particles in src order.
 *  *dst->d_count receives the output count and *d_uid_next [device] advances
 *  by it.  massive: 1 for leptons, 0 for photons.  src and dst are device
 *  species of one precision in distinct buffers, chi arrays both present or
 *  both NULL, dst->capacity >= src->capacity.  The merger holds 28 bytes per
 *  particle of scratch; calls on one workspace are ordered on one stream.
 *  QED_ERR_ARG: a null argument, nx ny nz below 1 or a product of 2^31 - 2
 *  or more, dx dy dz not > 0, n_octaves < 1, sub_bins not a power of two in
 *  1..64, n_dir outside 1..64, more than 2^31 momentum bins, min_group < 2,
 *  octave_min outside -1074..1023, mismatched or aliased species,
 *  src->capacity above the merger's maximum or the workspace's reach
 *  (4096 x its look-back tiles); QED_ERR_HIP if a launch fails.
 * ------------------------------------------------------------------------ */
typedef struct {
    double x0, y0, z0, dx, dy, dz;      /* box of cells                         */
    int64_t nx, ny, nz;
    int32_t massive;                    /* 1 leptons, 0 photons                 */
    int32_t octave_min, n_octaves;      /* energy range of |u|^2, in octaves    */
    int32_t sub_bins;                   /* energy bins per octave (power of 2)  */
    int32_t n_dir;                      /* direction bins per face edge         */
    int32_t min_group;                  /* merge groups of at least this many   */
} qed_merge_spec;

typedef struct qed_merger qed_merger;
qed_status qed_merger_create(int64_t max_particles, qed_merger **out);
void qed_merger_free(qed_merger *m);
qed_status qed_merge(qed_merger *m, qed_workspace *ws, const qed_merge_spec *spec, qed_species *src,
                     qed_species *dst, uint64_t seed, uint64_t *d_uid_next, void *stream);

/* ------------------------------------------------------------------------ *
 * Coupling to a particle-in-cell loop: the field solver and the currents.
 * The paper's PIC code advances Maxwell's equations and deposits currents
 * (Sec. 1, Sec. 3) without saying how; these are the textbook schemes.
 * Grids are FP32, component-major [c][nx][ny][nz] (z fastest), on the Yee
 * staggering of the field gather (Ex at (i+1/2, j, k), Bx at (i, j+1/2,
 * k+1/2), ...; J_c at the position of E_c), periodic in every direction.
 * The geometry comes from a qed_field of kind QED_FIELD_YEE (its grid
 * pointer is not used by the deposition calls).
 *
 * qed_yee_advance: Yee's scheme in normalised units (c = 1, fields in the
 *   units of the step): B -= (dt/2) curl E; E += dt curl B - dt J;
 *   B -= (dt/2) curl E, so that E and B are at whole steps.  J [device]
 *   3 n floats, or NULL for vacuum.  Each update is
 *   fmaf(c_a, d_a, fmaf(-c_b, d_b, fmaf(-dt, J, old))) with the
 *   coefficients rounded once to FP32, so results do not depend on the
 *   launch.  QED_ERR_ARG if dt is not below the Courant limit
 *   1/sqrt(1/dx^2 + 1/dy^2 + 1/dz^2).
 * qed_deposit_current: adds to J [device, 3 n floats] the charge-conserving
 *   current (Esirkepov, Comput. Phys. Commun. 135, 144 (2001)) of quadratic
 *   (TSC) particles [first, *s->d_count) moving over one step dt from
 *   (x_old, y_old, z_old)[p - first] [device, the species' precision] to
 *   their present position; x_old = NULL takes the start as x - dt u/gamma
 *   (particles created in the step).  first = *d_first [device], or 0 if
 *   d_first is NULL.  A particle of weight w adds node charges
 *   charge * w * j_scale * S_x S_y S_z (with w in physical particles,
 *   j_scale = 1/(n_c dx dy dz) in units of c/omega_r gives J in e n_c c).
 *   Particles whose nearest node moves by more than one cell along an axis
 *   are skipped and added to *d_skipped [device, may be NULL].  Decayed
 *   photons (tau = +INFINITY) are skipped silently.  Float atomics: the
 *   order of additions, and so the last bits of J, vary between runs.
 * qed_deposit_charge: adds the TSC node charges to rho [device, n floats].
 * qed_save_positions: copies x, y, z of entries [0, *d_count) to x_old,
 *   y_old, z_old [device, capacity entries of the species' precision].
 * ------------------------------------------------------------------------ */
qed_status qed_yee_advance(float *grid, const float *J, const qed_field *geometry, double dt, void *stream);
qed_status qed_deposit_current(const qed_species *s, const void *x_old, const void *y_old, const void *z_old,
                               const int64_t *d_first, double charge, double j_scale, double dt,
                               const qed_field *geometry, float *J, uint64_t *d_skipped, void *stream);
qed_status qed_deposit_charge(const qed_species *s, double charge, double j_scale, const qed_field *geometry,
                              float *rho, void *stream);
qed_status qed_save_positions(const qed_species *s, void *x_old, void *y_old, void *z_old, void *stream);

/* Advance a device step counter by one (for graph-captured step sequences). */
qed_status qed_step_advance(int64_t *d_step, void *stream);

#ifdef __cplusplus
}
#endif
#endif
