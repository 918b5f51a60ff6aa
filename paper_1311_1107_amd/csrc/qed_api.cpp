// qed_api.cpp -- the C interface declared in include/qed.h: argument checks,
// handle management and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qed.h"
#include "qed_kernels.h"
#include "qed_fields.h"
#include "qed_sort.h"

namespace qedtab {
int build_tables(double e_chi_min, double e_chi_max, int e_n_chi, int e_n_q, double e_logit,
                 double p_chi_min, double p_chi_max, int p_n_chi, int p_n_q, double p_logit,
                 double *ln_hrad, double *ln_g, double *emit_q, double *pair_lnh, double *pair_q);
void spline_quads(const double *q, int n_chi, int n_q, double h_c, double h_t, double *quad);
}

namespace {

thread_local std::string g_err;

qed_status fail(qed_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(QED_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool spec_ok(const qed_table_spec *s) {
    return s && s->n_chi >= 2 && s->n_chi <= qed::kMaxChiNodes && s->n_q >= 2 && s->n_q <= 256 &&
           s->chi_min > 0.0 && s->chi_max > s->chi_min && std::isfinite(s->chi_max) && s->logit_max > 0.0 &&
           (s->interp == QED_INTERP_LINEAR || s->interp == QED_INTERP_SPLINE) && s->reserved == 0;
}

}  // namespace

struct qed_tables {
    qed_table_spec emit, pair;
    int device;
    double *d64;      // ln_hrad | ln_g | emit_q | pair_lnh | pair_q
    float *d32;
    size_t off[6];    // element offsets of the five tables (and the total)
    double *s64;      // spline node quads (f, f_tt, f_cc, f_cctt): emission | pair
    float *s32;
    qed::TablesDev dev;
};

struct qed_sorter {
    int64_t max_particles;
    uint32_t *keys;               // 4 * max: key0, key1, idx0, idx1
    uint32_t *hist;               // 2 * 16 * tiles: histograms and their prefixes
    unsigned long long *live;
    int64_t hist_len;
};

struct qed_merger {
    int64_t max_particles;
    uint32_t *buf;                // 7 * max + 2: key0, key1, idx0, idx1, mkey, g (max + 1), o (max + 1)
    uint32_t *hist;               // 2 * hist_len
    int64_t *cnt;
    int64_t hist_len;
};

struct qed_workspace {
    int device;
    int n_cu;
    int64_t max_tiles;
    int64_t max_leptons;
    uint64_t *d_ticket;
    uint64_t *d_lb;
    unsigned long long *d_status;
    uint32_t *d_tiles;        // tile counts and prefixes, 4 * max_tiles
    qed::LaunchInfo *d_info;
    void *d_rec;              // emission records
    uint32_t *d_meta, *d_nrec;
    void *d_item;             // event items of the lepton step
    uint32_t *d_item_map;
    qed::WsDev dev;
};

extern "C" {

const char *qed_last_error(void) { return g_err.c_str(); }

qed_status qed_units_init(double lambda_m, qed_units *out) {
    if (!out || !(lambda_m > 0.0) || !std::isfinite(lambda_m)) return fail(QED_ERR_ARG, "qed_units_init: lambda must be > 0");
    // CODATA 2018 (exact SI definitions for c, e, h; measured m_e and eps0)
    const double c = 299792458.0, e = 1.602176634e-19, h = 6.62607015e-34;
    const double me = 9.1093837015e-31, eps0 = 8.8541878128e-12;
    const double hbar = h / (2.0 * qed::kPi);
    out->lambda = lambda_m;
    out->omega_r = 2.0 * qed::kPi * c / lambda_m;
    out->alpha_f = e * e / (4.0 * qed::kPi * eps0 * hbar * c);
    // E_s = m^2 c^3/(e hbar) over the field unit m c omega_r/e
    out->Es_hat = (me * c * c) / (hbar * out->omega_r);
    // alpha_f/(tau_c omega_r) with tau_c = hbar/(m c^2)
    out->A_hat = out->alpha_f * me * c * c / (hbar * out->omega_r);
    // tau_0 = 2 e^2/(12 pi eps0 m c^3)
    out->tau0_hat = 2.0 * e * e / (12.0 * qed::kPi * eps0 * me * c * c * c) * out->omega_r;
    return QED_OK;
}

// ------------------------------------------------------------------ tables --
qed_status qed_tables_compute_host(const qed_table_spec *emit, const qed_table_spec *pair,
                                   double *ln_hrad, double *ln_g, double *emit_q,
                                   double *pair_lnh, double *pair_q) {
    if (!spec_ok(emit) || !spec_ok(pair)) return fail(QED_ERR_ARG, "qed_tables_compute_host: invalid table spec");
    if (!ln_hrad || !ln_g || !emit_q || !pair_lnh || !pair_q) return fail(QED_ERR_ARG, "qed_tables_compute_host: null output");
    int rc = qedtab::build_tables(emit->chi_min, emit->chi_max, emit->n_chi, emit->n_q, emit->logit_max,
                                  pair->chi_min, pair->chi_max, pair->n_chi, pair->n_q, pair->logit_max,
                                  ln_hrad, ln_g, emit_q, pair_lnh, pair_q);
    if (rc) return fail(QED_ERR_RANGE, "qed_tables_compute_host: non-finite table entry");
    return QED_OK;
}

qed_status qed_tables_load(const qed_table_spec *emit, const qed_table_spec *pair,
                           const double *ln_hrad, const double *ln_g, const double *emit_q,
                           const double *pair_lnh, const double *pair_q, qed_tables **out) {
    if (!out) return fail(QED_ERR_ARG, "qed_tables_load: null out");
    *out = nullptr;
    if (!spec_ok(emit) || !spec_ok(pair)) return fail(QED_ERR_ARG, "qed_tables_load: invalid table spec");
    if (!ln_hrad || !ln_g || !emit_q || !pair_lnh || !pair_q) return fail(QED_ERR_ARG, "qed_tables_load: null input");
    qed_tables *t = new qed_tables();
    t->emit = *emit;
    t->pair = *pair;
    HIP_TRY(hipGetDevice(&t->device));
    const size_t ne = emit->n_chi, nq = emit->n_q, np = pair->n_chi, npq = pair->n_q;
    const size_t sizes[5] = {ne, ne, ne * nq, np, np * npq};
    t->off[0] = 0;
    for (int k = 0; k < 5; ++k) t->off[k + 1] = t->off[k] + sizes[k];
    const double *src[5] = {ln_hrad, ln_g, emit_q, pair_lnh, pair_q};
    std::vector<double> h64(t->off[5]);
    std::vector<float> h32(t->off[5]);
    for (int k = 0; k < 5; ++k)
        for (size_t j = 0; j < sizes[k]; ++j) {
            const double v = src[k][j];
            if (!std::isfinite(v)) { delete t; return fail(QED_ERR_ARG, "qed_tables_load: non-finite entry in table %d", k); }
            h64[t->off[k] + j] = v;
            h32[t->off[k] + j] = (float)v;
        }
    if (hipMalloc(&t->d64, sizeof(double) * t->off[5]) != hipSuccess ||
        hipMalloc(&t->d32, sizeof(float) * t->off[5]) != hipSuccess) {
        qed_tables_free(t);
        return fail(QED_ERR_NOMEM, "qed_tables_load: device allocation failed");
    }
    HIP_TRY(hipMemcpy(t->d64, h64.data(), sizeof(double) * t->off[5], hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t->d32, h32.data(), sizeof(float) * t->off[5], hipMemcpyHostToDevice));
    qed::TablesDev &d = t->dev;
    // spline form: each node of a quantile table as four adjacent values
    const double eh_c = (std::log(emit->chi_max) - std::log(emit->chi_min)) / (emit->n_chi - 1);
    const double eh_t = 2.0 * emit->logit_max / (emit->n_q - 1);
    const double ph_c = (std::log(pair->chi_max) - std::log(pair->chi_min)) / (pair->n_chi - 1);
    const double ph_t = 2.0 * pair->logit_max / (pair->n_q - 1);
    const size_t sq_e = emit->interp == QED_INTERP_SPLINE ? 4 * ne * nq : 0;
    const size_t sq_p = pair->interp == QED_INTERP_SPLINE ? 4 * np * npq : 0;
    if (sq_e + sq_p > 0) {
        std::vector<double> s64(sq_e + sq_p);
        if (sq_e) qedtab::spline_quads(emit_q, emit->n_chi, emit->n_q, eh_c, eh_t, s64.data());
        if (sq_p) qedtab::spline_quads(pair_q, pair->n_chi, pair->n_q, ph_c, ph_t, s64.data() + sq_e);
        std::vector<float> s32(s64.size());
        for (size_t k = 0; k < s64.size(); ++k) {
            if (!std::isfinite(s64[k])) { qed_tables_free(t); return fail(QED_ERR_ARG, "qed_tables_load: non-finite spline curvature"); }
            s32[k] = (float)s64[k];
        }
        if (hipMalloc(&t->s64, sizeof(double) * s64.size()) != hipSuccess ||
            hipMalloc(&t->s32, sizeof(float) * s32.size()) != hipSuccess) {
            qed_tables_free(t);
            return fail(QED_ERR_NOMEM, "qed_tables_load: device allocation failed");
        }
        HIP_TRY(hipMemcpy(t->s64, s64.data(), sizeof(double) * s64.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t->s32, s32.data(), sizeof(float) * s32.size(), hipMemcpyHostToDevice));
    }
    d.emit_qs = sq_e ? t->s64 : nullptr;
    d.emit_qs_f = sq_e ? t->s32 : nullptr;
    d.pair_qs = sq_p ? t->s64 + sq_e : nullptr;
    d.pair_qs_f = sq_p ? t->s32 + sq_e : nullptr;
    d.e_ht26 = eh_t * eh_t / 6.0; d.e_hc26 = eh_c * eh_c / 6.0;
    d.p_ht26 = ph_t * ph_t / 6.0; d.p_hc26 = ph_c * ph_c / 6.0;
    d.ln_hrad = t->d64 + t->off[0]; d.ln_g = t->d64 + t->off[1]; d.emit_q = t->d64 + t->off[2];
    d.pair_lnh = t->d64 + t->off[3]; d.pair_q = t->d64 + t->off[4];
    d.ln_hrad_f = t->d32 + t->off[0]; d.ln_g_f = t->d32 + t->off[1]; d.emit_q_f = t->d32 + t->off[2];
    d.pair_lnh_f = t->d32 + t->off[3]; d.pair_q_f = t->d32 + t->off[4];
    d.e_n_chi = emit->n_chi; d.e_n_q = emit->n_q; d.p_n_chi = pair->n_chi; d.p_n_q = pair->n_q;
    d.e_chi_min = emit->chi_min;
    d.e_inv_chi_min = 1.0 / emit->chi_min;
    d.e_h0 = std::exp(ln_hrad[0]);
    d.e_lnchi0 = std::log(emit->chi_min);
    d.e_inv_dlnchi = (emit->n_chi - 1) / (std::log(emit->chi_max) - std::log(emit->chi_min));
    d.e_logit_max = emit->logit_max;
    d.e_inv_dt = (emit->n_q - 1) / (2.0 * emit->logit_max);
    d.p_chi_min = pair->chi_min;
    d.p_lnchi0 = std::log(pair->chi_min);
    d.p_inv_dlnchi = (pair->n_chi - 1) / (std::log(pair->chi_max) - std::log(pair->chi_min));
    d.p_logit_max = pair->logit_max;
    d.p_inv_dt = (pair->n_q - 1) / (2.0 * pair->logit_max);
    *out = t;
    return QED_OK;
}

qed_status qed_tables_build(const qed_table_spec *emit, const qed_table_spec *pair, qed_tables **out) {
    if (!out) return fail(QED_ERR_ARG, "qed_tables_build: null out");
    *out = nullptr;
    if (!spec_ok(emit) || !spec_ok(pair)) return fail(QED_ERR_ARG, "qed_tables_build: invalid table spec");
    std::vector<double> a(emit->n_chi), b(emit->n_chi), c((size_t)emit->n_chi * emit->n_q),
        d(pair->n_chi), e((size_t)pair->n_chi * pair->n_q);
    qed_status st = qed_tables_compute_host(emit, pair, a.data(), b.data(), c.data(), d.data(), e.data());
    if (st != QED_OK) return st;
    return qed_tables_load(emit, pair, a.data(), b.data(), c.data(), d.data(), e.data(), out);
}

qed_status qed_tables_export(const qed_tables *t, int32_t which, double *host, size_t n) {
    if (!t || !host || which < 0 || which > 4) return fail(QED_ERR_ARG, "qed_tables_export: bad arguments");
    const size_t len = t->off[which + 1] - t->off[which];
    if (n != len) return fail(QED_ERR_ARG, "qed_tables_export: table %d has %zu entries, not %zu", which, len, n);
    HIP_TRY(hipMemcpy(host, t->d64 + t->off[which], sizeof(double) * len, hipMemcpyDeviceToHost));
    return QED_OK;
}

void qed_tables_free(qed_tables *t) {
    if (!t) return;
    (void)hipFree(t->d64);
    (void)hipFree(t->d32);
    (void)hipFree(t->s64);
    (void)hipFree(t->s32);
    delete t;
}

// --------------------------------------------------------------- workspace --
qed_status qed_workspace_create(int64_t max_particles, int64_t max_leptons, qed_workspace **out) {
    if (!out) return fail(QED_ERR_ARG, "qed_workspace_create: null out");
    *out = nullptr;
    if (max_particles < 1 || max_particles > (int64_t)1 << 40 || max_leptons < 0 || max_leptons > max_particles)
        return fail(QED_ERR_ARG, "qed_workspace_create: need 1 <= max_particles <= 2^40, 0 <= max_leptons <= max_particles");
    qed_workspace *w = new qed_workspace();
    HIP_TRY(hipGetDevice(&w->device));
    HIP_TRY(hipDeviceGetAttribute(&w->n_cu, hipDeviceAttributeMultiprocessorCount, w->device));
    // smallest tile is 64 threads x 1 particle
    // rounded up to 16 tiles so that every per-tile array starts 64-byte aligned (wide loads in the scans)
    w->max_tiles = ((max_particles + 63) / 64 + 1 + 15) / 16 * 16;
    w->max_leptons = max_leptons;
    if (w->max_tiles > 0xffffffffll) { delete w; return fail(QED_ERR_ARG, "qed_workspace_create: too many tiles"); }
    const int64_t slots = ((max_leptons + 255) / 256 + 1) * 256;
    if (hipMalloc(&w->d_ticket, 64) != hipSuccess || hipMalloc(&w->d_lb, sizeof(uint64_t) * 4 * w->max_tiles) != hipSuccess ||
        hipMalloc(&w->d_status, 64) != hipSuccess || hipMalloc(&w->d_tiles, sizeof(uint32_t) * 4 * w->max_tiles) != hipSuccess ||
        hipMalloc(&w->d_info, sizeof(qed::LaunchInfo)) != hipSuccess ||
        hipMalloc(&w->d_rec, sizeof(double) * qed::kRecReals * slots) != hipSuccess ||
        hipMalloc(&w->d_meta, sizeof(uint32_t) * slots) != hipSuccess ||
        hipMalloc(&w->d_nrec, sizeof(uint32_t) * w->max_tiles) != hipSuccess ||
        hipMalloc(&w->d_item, qed::kItemBytes * slots) != hipSuccess ||
        hipMalloc(&w->d_item_map, sizeof(uint32_t) * slots) != hipSuccess) {
        qed_workspace_free(w);
        return fail(QED_ERR_NOMEM, "qed_workspace_create: device allocation failed");
    }
    // epoch 1 in the ticket's high word: zeroed look-back words (epoch 0) never match
    const uint64_t ticket0[8] = {1ull << 32, 0, 0, 0, 0, 0, 0, 0};
    std::vector<uint64_t> zeros(4 * w->max_tiles, 0ull);
    HIP_TRY(hipMemcpy(w->d_ticket, ticket0, 64, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_lb, zeros.data(), sizeof(uint64_t) * 4 * w->max_tiles, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_status, zeros.data(), 64, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_nrec, zeros.data(), sizeof(uint32_t) * w->max_tiles, hipMemcpyHostToDevice));
    w->dev.ticket = w->d_ticket;
    w->dev.lb.agg0 = w->d_lb;
    w->dev.lb.agg1 = w->d_lb + w->max_tiles;
    w->dev.lb.inc0 = w->d_lb + 2 * w->max_tiles;
    w->dev.lb.inc1 = w->d_lb + 3 * w->max_tiles;
    w->dev.status = w->d_status;
    w->dev.tile_cnt0 = w->d_tiles;
    w->dev.tile_cnt1 = w->d_tiles + w->max_tiles;
    w->dev.tile_pre0 = w->d_tiles + 2 * w->max_tiles;
    w->dev.tile_pre1 = w->d_tiles + 3 * w->max_tiles;
    w->dev.info = w->d_info;
    w->dev.stage.rec = w->d_rec;
    w->dev.stage.meta = w->d_meta;
    w->dev.stage.n_rec = w->d_nrec;
    w->dev.stage.item = w->d_item;
    w->dev.stage.item_map = w->d_item_map;
    w->dev.stage.slots = slots;
    w->dev.max_tiles = w->max_tiles;
    *out = w;
    return QED_OK;
}

void qed_workspace_free(qed_workspace *w) {
    if (!w) return;
    (void)hipFree(w->d_ticket);
    (void)hipFree(w->d_lb);
    (void)hipFree(w->d_status);
    (void)hipFree(w->d_tiles);
    (void)hipFree(w->d_info);
    (void)hipFree(w->d_rec);
    (void)hipFree(w->d_meta);
    (void)hipFree(w->d_nrec);
    (void)hipFree(w->d_item);
    (void)hipFree(w->d_item_map);
    delete w;
}

qed_status qed_sync_status(qed_workspace *w, qed_status_report *out, int32_t clear, void *stream) {
    if (!w || !out) return fail(QED_ERR_ARG, "qed_sync_status: null argument");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long h[8];
    HIP_TRY(hipMemcpy(h, w->d_status, 64, hipMemcpyDeviceToHost));
    out->flags = (int64_t)h[0];
    for (int k = 0; k < 4; ++k) out->needed[k] = (int64_t)h[1 + k];
    out->chi_above_table = (int64_t)h[5];
    if (clear) {
        const unsigned long long z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        HIP_TRY(hipMemcpy(w->d_status, z, 64, hipMemcpyHostToDevice));
    }
    if (h[0] & 1ull) return fail(QED_ERR_CAPACITY, "an append did not fit its buffer (needed %lld/%lld/%lld/%lld)",
                                 (long long)h[1], (long long)h[2], (long long)h[3], (long long)h[4]);
    if (h[0] & 2ull) return fail(QED_ERR_RANGE, "non-finite particle state met on the device");
    return QED_OK;
}

qed_status qed_tally_reduce(const qed_tally *t, double energy[QED_N_ENERGY], int64_t count[QED_N_COUNT],
                            void *stream) {
    if (!t || !t->energy || !t->count || t->n_slots < 1 || !energy || !count)
        return fail(QED_ERR_ARG, "qed_tally_reduce: bad arguments");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    std::vector<double> e((size_t)t->n_slots * QED_N_ENERGY);
    HIP_TRY(hipMemcpy(e.data(), t->energy, sizeof(double) * e.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(count, t->count, sizeof(int64_t) * QED_N_COUNT, hipMemcpyDeviceToHost));
    for (int k = 0; k < QED_N_ENERGY; ++k) {
        double s = 0.0;
        for (int64_t j = 0; j < t->n_slots; ++j) s += e[(size_t)j * QED_N_ENERGY + k];
        energy[k] = s;
    }
    return QED_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ checks --
namespace {

qed_status species_dev(const qed_species *s, bool need_chi, const char *what, qed::SpeciesDev &d) {
    std::memset(&d, 0, sizeof d);
    if (!s) return QED_OK;
    if (s->prec != QED_F64 && s->prec != QED_F32) return fail(QED_ERR_ARG, "%s: prec must be QED_F64 or QED_F32", what);
    if (!s->x || !s->y || !s->z || !s->ux || !s->uy || !s->uz || !s->tau || !s->w || !s->uid || !s->n_event || !s->d_count)
        return fail(QED_ERR_ARG, "%s: null array", what);
    if (need_chi && !s->chi) return fail(QED_ERR_ARG, "%s: photons need the chi array", what);
    if (s->capacity < 0 || s->capacity > 0xffffffffll * 64) return fail(QED_ERR_ARG, "%s: bad capacity", what);
    d.x = s->x; d.y = s->y; d.z = s->z; d.ux = s->ux; d.uy = s->uy; d.uz = s->uz;
    d.tau = s->tau; d.w = s->w; d.chi = s->chi; d.uid = s->uid; d.n_ev = s->n_event;
    d.count = s->d_count; d.cap = s->capacity; d.present = 1;
    return QED_OK;
}

qed_status field_dev(const qed_field *f, int prec, qed::FieldDev &d, int &fk) {
    std::memset(&d, 0, sizeof d);
    if (!f) return fail(QED_ERR_ARG, "field: null");
    d.kind = f->kind;
    for (int c = 0; c < 3; ++c) { d.E[c] = f->E[c]; d.B[c] = f->B[c]; }
    if (f->kind == QED_FIELD_UNIFORM) {
        fk = qed::FIELD_UNIFORM;
    } else if (f->kind == QED_FIELD_PLANE_WAVE) {
        if (!(f->n_periods > 0.0) || !std::isfinite(f->a0)) return fail(QED_ERR_ARG, "field: plane wave needs n_periods > 0");
        d.a0 = f->a0;
        d.Phi = 2.0 * qed::kPi * f->n_periods;
        d.inv_Phi = 1.0 / d.Phi;
        fk = qed::FIELD_PLANE;
    } else if (f->kind == QED_FIELD_YEE) {
        if (!f->grid || f->nx < 1 || f->ny < 1 || f->nz < 1 || !(f->dx > 0) || !(f->dy > 0) || !(f->dz > 0))
            return fail(QED_ERR_ARG, "field: Yee grid needs a grid pointer, sizes and spacings");
        d.grid = f->grid; d.nx = f->nx; d.ny = f->ny; d.nz = f->nz;
        d.inv_dx = 1.0 / f->dx; d.inv_dy = 1.0 / f->dy; d.inv_dz = 1.0 / f->dz;
        d.x0 = f->x0; d.y0 = f->y0; d.z0 = f->z0;
        if (f->bound) {
            if (f->bound_block < 1 || f->bound_block > 64)
                return fail(QED_ERR_ARG, "field: bound_block must be in 1..64 with a bound table");
            d.bound = f->bound;
            d.bb = f->bound_block;
            d.nbx = (f->nx + d.bb - 1) / d.bb; d.nby = (f->ny + d.bb - 1) / d.bb; d.nbz = (f->nz + d.bb - 1) / d.bb;
        }
        fk = qed::FIELD_YEE;
    } else {
        return fail(QED_ERR_ARG, "field: unknown kind %d", f->kind);
    }
    (void)prec;
    return QED_OK;
}

qed_status step_dev(const qed_step *s, qed::StepDev &d) {
    if (!s) return fail(QED_ERR_ARG, "step: null");
    if (!(s->dt > 0.0) || !std::isfinite(s->t)) return fail(QED_ERR_ARG, "step: dt must be > 0 and t finite");
    if (s->rad_model < QED_RAD_NONE || s->rad_model > QED_RAD_HYBRID) return fail(QED_ERR_ARG, "step: bad rad_model");
    if (s->max_events < 1 || s->max_events > qed::kMaxEvents) return fail(QED_ERR_ARG, "step: max_events must be 1..4");
    d.t = s->t; d.dt = s->dt; d.d_step = s->d_step; d.seed = s->seed;
    d.rad = s->rad_model; d.kmax = s->max_events; d.chi_switch = s->chi_switch;
    d.gmin = s->gamma_photon_min; d.chi_push_min = s->chi_photon_push_min; d.no_recoil = s->no_recoil;
    if (s->variants & ~(QED_VAR_SOKOLOV_G | QED_VAR_PAIR_MOMENTUM)) return fail(QED_ERR_ARG, "step: unknown variant bits");
    d.variants = s->variants;
    return QED_OK;
}

qed_status tally_dev(const qed_tally *t, qed::TallyDev &d) {
    if (!t || !t->energy || !t->count || t->n_slots < 1) return fail(QED_ERR_ARG, "tally: needs energy, count and n_slots >= 1");
    d.energy = t->energy; d.count = t->count; d.n_slots = t->n_slots;
    return QED_OK;
}

qed_status consts_dev(const qed_units *u, double q, qed::ConstsDev &c) {
    if (!u || !(u->Es_hat > 0) || !(u->A_hat > 0) || !(u->tau0_hat >= 0)) return fail(QED_ERR_ARG, "units: invalid");
    c.q = q; c.es_inv = 1.0 / u->Es_hat; c.A = u->A_hat; c.tau0 = u->tau0_hat;
    return QED_OK;
}

// Launch shape of the physics passes: a persistent grid whose size is a
// multiple of 8 (one share per XCD).
// What the launches need to know of a workspace: the device view, the CU
// count for the grid and the limits of its per-tile arrays and staging.
struct WsInfo {
    qed::WsDev dev;
    int n_cu;
    int64_t max_tiles, max_leptons;
};

WsInfo info_of(const qed_workspace *w) {
    return WsInfo{w->dev, w->n_cu, w->max_tiles, w->max_leptons};
}

qed_status shape(const WsInfo &w, const qed_schedule *s, int64_t capacity, dim3 &grid, dim3 &block) {
    int b = 256, ipt = 1, bpc = 8, cap = 0;
    if (s) {
        if (s->block) b = s->block;
        if (s->items_per_thread) ipt = s->items_per_thread;
        if (s->blocks_per_cu) bpc = s->blocks_per_cu;
        cap = s->max_blocks;
    }
    if (b < 64 || b > 256 || b % 64) return fail(QED_ERR_ARG, "schedule: block must be 64, 128, 192 or 256");
    if (ipt != 1) return fail(QED_ERR_ARG, "schedule: items_per_thread must be 1");
    if (bpc < 1 || bpc > 64) return fail(QED_ERR_ARG, "schedule: blocks_per_cu must be 1..64");
    if (cap != 0 && cap < 8) return fail(QED_ERR_ARG, "schedule: max_blocks must be 0 or at least 8");
    const int64_t tiles = (capacity + b - 1) / b;
    if (tiles + 1 > w.max_tiles) return fail(QED_ERR_ARG, "workspace too small for %lld particles", (long long)capacity);
    int64_t g = (int64_t)w.n_cu * bpc;
    g = std::min<int64_t>(g, ((tiles + 7) / 8) * 8);
    if (cap) g = std::min<int64_t>(g, cap);
    g = std::max<int64_t>(8, (g / 8) * 8);
    grid = dim3((unsigned)g);
    block = dim3((unsigned)b);
    return QED_OK;
}

// Grid of the scan pass: one block per 4096 tile counts, at most one per CU.
dim3 scan_grid(const WsInfo &w, int64_t capacity, int64_t tile_sz) {
    const int64_t tiles = (capacity + tile_sz - 1) / tile_sz;
    const int64_t blocks = (tiles + 4095) / 4096;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, w.n_cu)));
}

}  // namespace

extern "C" {

qed_status qed_init_optical_depth(qed_species *s, uint64_t seed, void *stream) {
    qed::SpeciesDev d;
    if (!s) return fail(QED_ERR_ARG, "qed_init_optical_depth: null species");
    qed_status st = species_dev(s, false, "qed_init_optical_depth", d);
    if (st) return st;
    int nb = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (s->capacity + 255) / 256));
    HIP_TRY(qed::launch_init_tau(s->uid, s->tau, s->d_count, seed, nb, (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_yee_fill_separable(float *grid, int64_t nx, int64_t ny, int64_t nz, double a0,
                                  const double *tperp, const double *tpar, void *stream) {
    if (!grid || !tperp || !tpar || nx < 1 || ny < 1 || nz < 1) return fail(QED_ERR_ARG, "qed_yee_fill_separable: bad arguments");
    const int64_t total = 6 * nx * ny * nz;
    int nb = (int)std::min<int64_t>(65536, (total + 255) / 256);
    HIP_TRY(qed::launch_yee_fill(grid, nx, ny, nz, a0, tperp, tpar, nb, (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_spectrum(const qed_species *s, int32_t photons, double e_min, double e_max, int32_t n_bins,
                        double weight_scale, int64_t *count, int64_t *wsum, void *stream) {
    if (!s || !count || !wsum) return fail(QED_ERR_ARG, "qed_spectrum: null argument");
    if (n_bins < 1 || n_bins > 1024) return fail(QED_ERR_ARG, "qed_spectrum: n_bins must be 1..1024");
    if (!(e_min > 0.0) || !(e_max > e_min) || !std::isfinite(e_max))
        return fail(QED_ERR_ARG, "qed_spectrum: need 0 < e_min < e_max");
    if (!(weight_scale > 0.0) || !std::isfinite(weight_scale)) return fail(QED_ERR_ARG, "qed_spectrum: weight_scale must be > 0");
    qed::SpectrumArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status st = species_dev(s, false, "qed_spectrum", a.s);
    if (st) return st;
    a.photons = photons ? 1 : 0;
    a.n_bins = n_bins;
    a.e_min = e_min;
    a.e_max = e_max;
    a.ln_emin = std::log(e_min);
    a.inv_dln = (double)n_bins / std::log(e_max / e_min);
    a.wscale = weight_scale;
    a.count = (unsigned long long *)count;
    a.wsum = (unsigned long long *)wsum;
    const int nb = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (s->capacity + 255) / 256));
    HIP_TRY(qed::launch_spectrum(a, s->prec, nb, (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_step_advance(int64_t *d_step, void *stream) {
    if (!d_step) return fail(QED_ERR_ARG, "qed_step_advance: null counter");
    HIP_TRY(qed::launch_step_advance(d_step, (hipStream_t)stream));
    return QED_OK;
}

static qed_status push_common(const qed_tables *tab, const WsInfo &ws, const qed_units *u, double charge,
                              qed_species *lep, qed::FieldDev &fd, int fk, qed_species *pp, qed_species *pr,
                              qed_tally *tally, const qed_step *st, uint64_t *uid_next, const qed_schedule *sched,
                              void *stream) {
    if (!tab || !lep || !uid_next) return fail(QED_ERR_ARG, "qed_push_emit: null argument");
    if (charge != -1.0 && charge != 1.0) return fail(QED_ERR_ARG, "qed_push_emit: charge must be -1 or +1");
    qed::PushArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status s;
    if ((s = species_dev(lep, false, "qed_push_emit(leptons)", a.lep))) return s;
    if ((s = species_dev(pp, true, "qed_push_emit(pushed photons)", a.pp))) return s;
    if ((s = species_dev(pr, true, "qed_push_emit(recorded photons)", a.pr))) return s;
    if ((pp && pp->prec != lep->prec) || (pr && pr->prec != lep->prec))
        return fail(QED_ERR_ARG, "qed_push_emit: photons and leptons must share a precision");
    if ((s = step_dev(st, a.st))) return s;
    if ((s = tally_dev(tally, a.tal))) return s;
    if ((s = consts_dev(u, charge, a.c))) return s;
    a.tab = tab->dev;
    a.f = fd;
    a.ws = ws.dev;
    a.uid_next = uid_next;
    if (lep->capacity > ws.max_leptons)
        return fail(QED_ERR_ARG, "qed_push_emit: %lld leptons exceed the workspace's max_leptons %lld",
                    (long long)lep->capacity, (long long)ws.max_leptons);
    if (lep->capacity >= ((int64_t)1 << 32))
        return fail(QED_ERR_ARG, "qed_push_emit: lepton capacity must be below 2^32");
    dim3 grid, block;
    if ((s = shape(ws, sched, lep->capacity, grid, block))) return s;
    a.tile_sz = qed::kWave;
    hipStream_t st_ = (hipStream_t)stream;
    // stream pass (tiles of one wave); list of the particles with events; event
    // pass over that list in full waves; scan of the photon counts per 64
    // events; photon appends
    HIP_TRY(qed::launch_lepton_stream(a, lep->prec, fk, grid, block, st_));
    qed::ScanArgs sc;
    std::memset(&sc, 0, sizeof sc);
    sc.src_count = lep->d_count;
    sc.tile_sz = qed::kWave;
    sc.uid_next = uid_next;                  // not read in this mode
    sc.mode = 2;
    sc.ws = ws.dev;
    const dim3 sg = scan_grid(ws, lep->capacity, qed::kWave);
    HIP_TRY(qed::launch_scan_tiles(sc, sg, st_));
    HIP_TRY(qed::launch_lepton_events(a, lep->prec, grid, block, st_));
    std::memset(&sc, 0, sizeof sc);
    sc.src_count = &ws.dev.info->n_items;
    sc.tile_sz = qed::kWave;
    sc.d0 = a.pp;
    sc.d1 = a.pr;
    sc.uid_next = uid_next;
    sc.mode = 0;
    sc.ws = ws.dev;
    HIP_TRY(qed::launch_scan_tiles(sc, sg, st_));
    HIP_TRY(qed::launch_push_append(a, lep->prec, grid, dim3(256), st_));
    return QED_OK;
}

qed_status qed_push_emit(const qed_tables *tab, qed_workspace *ws, const qed_units *u, double charge,
                         qed_species *lep, const qed_field *f, qed_species *ph_push, qed_species *ph_rec,
                         qed_tally *tally, const qed_step *st, uint64_t *d_uid_next, const qed_schedule *sched,
                         void *stream) {
    if (!lep) return fail(QED_ERR_ARG, "qed_push_emit: null leptons");
    qed::FieldDev fd;
    int fk = 0;
    qed_status s = field_dev(f, lep->prec, fd, fk);
    if (s) return s;
    if (!ws) return fail(QED_ERR_ARG, "qed_push_emit: null workspace");
    return push_common(tab, info_of(ws), u, charge, lep, fd, fk, ph_push, ph_rec, tally, st, d_uid_next, sched, stream);
}

qed_status qed_push_emit_batched(const qed_tables *tab, qed_workspace *ws, const qed_units *u, double charge,
                                 qed_species *lep, const qed_bunches *b, qed_species *ph_push, qed_species *ph_rec,
                                 qed_tally *tally, const qed_step *st, uint64_t *d_uid_next,
                                 const qed_schedule *sched, void *stream) {
    if (!b || b->n_bunches < 1 || !b->offsets || !b->a0 || !b->n_periods)
        return fail(QED_ERR_ARG, "qed_push_emit_batched: bad bunch table");
    qed::FieldDev fd;
    std::memset(&fd, 0, sizeof fd);
    fd.kind = -1;
    fd.n_bunches = b->n_bunches;
    fd.offsets = b->offsets;
    fd.a0s = b->a0;
    fd.nper = b->n_periods;
    fd.lds_bunches = qed::lds_bunch_bytes(b->n_bunches) <= qed::kLdsBunchBytes;
    if (!ws) return fail(QED_ERR_ARG, "qed_push_emit_batched: null workspace");
    return push_common(tab, info_of(ws), u, charge, lep, fd, qed::FIELD_BUNCHED, ph_push, ph_rec, tally, st,
                       d_uid_next, sched, stream);
}

}  // extern "C"

// ---------------------------------------------------- static scratch -------
// qed_push_emit_static keeps the lepton step's scratch (look-back words,
// per-tile counts and prefixes, emission records, ticket and status) in one
// file-scope device array instead of a qed_workspace, for callers that cannot
// allocate.  Each device holds its own copy until the process ends.  Host
// code never uses the array's name for its memory: the address comes from
// hipGetSymbolAddress, once per device.
namespace {

constexpr int64_t kStaticMaxLeptons = 65536;                       // per call
constexpr int64_t kStaticTiles = (kStaticMaxLeptons / 64 + 1 + 15) / 16 * 16;  // tiles of 64, rounded to 16
constexpr int64_t kStaticSlots = ((kStaticMaxLeptons + 255) / 256 + 1) * 256;

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffTicket = 0;
constexpr size_t kOffStatus = 256;
constexpr size_t kOffInfo = 512;
constexpr size_t kOffLb = 768;
constexpr size_t kOffTiles = kOffLb + align256(sizeof(uint64_t) * 4 * kStaticTiles);
constexpr size_t kOffNrec = kOffTiles + align256(sizeof(uint32_t) * 4 * kStaticTiles);
constexpr size_t kOffMeta = kOffNrec + align256(sizeof(uint32_t) * kStaticTiles);
constexpr size_t kOffRec = kOffMeta + align256(sizeof(uint32_t) * kStaticSlots);
constexpr size_t kOffItem = kOffRec + align256(sizeof(double) * qed::kRecReals * kStaticSlots);
constexpr size_t kOffItemMap = kOffItem + align256(qed::kItemBytes * kStaticSlots);
constexpr size_t kStaticBytes = kOffItemMap + align256(sizeof(uint32_t) * kStaticSlots);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
unsigned char *g_static_ptr[kMaxDevices];      // device address of `scratch`, per device
int g_static_ncu[kMaxDevices];

// First use on a device: zero the status and the look-back words and put the
// ticket at epoch 1 (zeroed look-back words, epoch 0, never match).  Runs
// only while the ticket is still zero, so running it again (a replayed
// graph) changes nothing.
__global__ void __launch_bounds__(1024) k_static_init(unsigned char *base) {
    __shared__ int s_fresh;
    uint64_t *ticket = (uint64_t *)(base + kOffTicket);
    if (threadIdx.x == 0) s_fresh = *ticket == 0ull;
    __syncthreads();
    if (!s_fresh) return;
    unsigned long long *st = (unsigned long long *)(base + kOffStatus);
    uint64_t *lb = (uint64_t *)(base + kOffLb);
    for (int64_t i = threadIdx.x; i < 4 * kStaticTiles; i += blockDim.x) lb[i] = 0ull;
    if (threadIdx.x < 8) st[threadIdx.x] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        *ticket = 1ull << 32;
    }
}

// The call's device status into the caller's words (flags OR'ed, needed
// counts raised to the largest), then the static status cleared.
__global__ void k_static_status(unsigned char *base, unsigned long long *out) {
    unsigned long long *st = (unsigned long long *)(base + kOffStatus);
    const int k = threadIdx.x;
    if (k < 6) {
        const unsigned long long v = st[k];
        if (k == 0) out[0] |= v;
        else if (v > out[k]) out[k] = v;
        st[k] = 0ull;
    }
}

qed_status static_scratch(int device, unsigned char **ptr, int *n_cu) {
    if (device < 0 || device >= kMaxDevices) return fail(QED_ERR_ARG, "qed_push_emit_static: device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(QED_ERR_HIP, "qed_push_emit_static: no address for the static scratch");
        HIP_TRY(hipDeviceGetAttribute(&g_static_ncu[device], hipDeviceAttributeMultiprocessorCount, device));
        hipLaunchKernelGGL(k_static_init, dim3(1), dim3(1024), 0, (hipStream_t)0, (unsigned char *)p);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipDeviceSynchronize());
        g_static_ptr[device] = (unsigned char *)p;
    }
    *ptr = g_static_ptr[device];
    *n_cu = g_static_ncu[device];
    return QED_OK;
}

}  // namespace

extern "C" {

qed_status qed_push_emit_static(const qed_tables *tab, const qed_units *u, double charge, qed_species *lep,
                                const qed_field *f, qed_species *ph_push, qed_species *ph_rec, qed_tally *tally,
                                const qed_step *st, uint64_t *d_uid_next, uint64_t *d_status,
                                const qed_schedule *sched, void *stream) {
    if (!lep || !d_status) return fail(QED_ERR_ARG, "qed_push_emit_static: null leptons or status words");
    if (lep->capacity > kStaticMaxLeptons)
        return fail(QED_ERR_ARG, "qed_push_emit_static: lepton capacity %lld exceeds the static scratch limit of %lld",
                    (long long)lep->capacity, (long long)kStaticMaxLeptons);
    qed::FieldDev fd;
    int fk = 0;
    qed_status s = field_dev(f, lep->prec, fd, fk);
    if (s) return s;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    unsigned char *base = nullptr;
    int n_cu = 0;
    if ((s = static_scratch(device, &base, &n_cu))) return s;
    WsInfo w;
    std::memset(&w, 0, sizeof w);
    w.n_cu = n_cu;
    w.max_tiles = kStaticTiles;
    w.max_leptons = kStaticMaxLeptons;
    uint64_t *lb = (uint64_t *)(base + kOffLb);
    uint32_t *tiles = (uint32_t *)(base + kOffTiles);
    w.dev.ticket = (uint64_t *)(base + kOffTicket);
    w.dev.lb.agg0 = lb;
    w.dev.lb.agg1 = lb + kStaticTiles;
    w.dev.lb.inc0 = lb + 2 * kStaticTiles;
    w.dev.lb.inc1 = lb + 3 * kStaticTiles;
    w.dev.status = (unsigned long long *)(base + kOffStatus);
    w.dev.tile_cnt0 = tiles;
    w.dev.tile_cnt1 = tiles + kStaticTiles;
    w.dev.tile_pre0 = tiles + 2 * kStaticTiles;
    w.dev.tile_pre1 = tiles + 3 * kStaticTiles;
    w.dev.info = (qed::LaunchInfo *)(base + kOffInfo);
    w.dev.stage.rec = base + kOffRec;
    w.dev.stage.meta = (uint32_t *)(base + kOffMeta);
    w.dev.stage.n_rec = (uint32_t *)(base + kOffNrec);
    w.dev.stage.item = base + kOffItem;
    w.dev.stage.item_map = (uint32_t *)(base + kOffItemMap);
    w.dev.stage.slots = kStaticSlots;
    w.dev.max_tiles = kStaticTiles;
    if ((s = push_common(tab, w, u, charge, lep, fd, fk, ph_push, ph_rec, tally, st, d_uid_next, sched, stream)))
        return s;
    hipLaunchKernelGGL(k_static_status, dim3(1), dim3(64), 0, (hipStream_t)stream, base,
                       (unsigned long long *)d_status);
    HIP_TRY(hipGetLastError());
    return QED_OK;
}

qed_status qed_pair_create(const qed_tables *tab, qed_workspace *ws, const qed_units *u, qed_species *ph,
                           const qed_field *f, qed_species *elec, qed_species *posi, qed_tally *tally,
                           const qed_step *st, uint64_t *d_uid_next, const qed_schedule *sched, void *stream) {
    if (!tab || !ws || !ph || !elec || !posi || !d_uid_next) return fail(QED_ERR_ARG, "qed_pair_create: null argument");
    qed::PairArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status s;
    if ((s = species_dev(ph, true, "qed_pair_create(photons)", a.ph))) return s;
    if ((s = species_dev(elec, false, "qed_pair_create(electrons)", a.el))) return s;
    if ((s = species_dev(posi, false, "qed_pair_create(positrons)", a.po))) return s;
    if (elec->prec != ph->prec || posi->prec != ph->prec) return fail(QED_ERR_ARG, "qed_pair_create: mixed precisions");
    int fk = 0;
    if ((s = field_dev(f, ph->prec, a.f, fk))) return s;
    if ((s = step_dev(st, a.st))) return s;
    if ((s = tally_dev(tally, a.tal))) return s;
    if ((s = consts_dev(u, 0.0, a.c))) return s;
    a.tab = tab->dev;
    a.ws = ws->dev;
    a.uid_next = d_uid_next;
    dim3 grid, block;
    if ((s = shape(info_of(ws), sched, ph->capacity, grid, block))) return s;
    // the physics pass counts pairs per wave (tiles of 64 photons)
    const int64_t tile_sz = 64;
    if ((ph->capacity + tile_sz - 1) / tile_sz + 1 > ws->max_tiles)
        return fail(QED_ERR_ARG, "qed_pair_create: workspace too small for %lld photons", (long long)ph->capacity);
    a.tile_sz = tile_sz;
    hipStream_t st_ = (hipStream_t)stream;
    // physics pass, scan of the per-tile pair counts, pair appends
    HIP_TRY(qed::launch_pair_create(a, ph->prec, fk, grid, block, st_));
    qed::ScanArgs sc;
    std::memset(&sc, 0, sizeof sc);
    sc.src_count = ph->d_count;
    sc.tile_sz = tile_sz;
    sc.d0 = a.el;
    sc.d1 = a.po;
    sc.uid_next = d_uid_next;
    sc.mode = 1;
    sc.ws = ws->dev;
    HIP_TRY(qed::launch_scan_tiles(sc, scan_grid(info_of(ws), ph->capacity, tile_sz), st_));
    HIP_TRY(qed::launch_pair_append(a, ph->prec, fk, grid, dim3(256), st_));
    return QED_OK;
}

qed_status qed_compact(qed_workspace *ws, qed_species *ph, const qed_schedule *sched, void *stream) {
    if (!ws || !ph) return fail(QED_ERR_ARG, "qed_compact: null argument");
    qed::CompactArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status s;
    if ((s = species_dev(ph, false, "qed_compact", a.s))) return s;
    a.ws = ws->dev;
    dim3 grid, block;
    if ((s = shape(info_of(ws), sched, ph->capacity, grid, block))) return s;
    HIP_TRY(qed::launch_compact(a, ph->prec, grid, block, (hipStream_t)stream));
    return QED_OK;
}

// -------------------------------------------------------------- cell sort --
qed_status qed_sorter_create(int64_t max_particles, qed_sorter **out) {
    if (!out) return fail(QED_ERR_ARG, "qed_sorter_create: null out");
    *out = nullptr;
    if (max_particles < 1 || max_particles >= (int64_t)0xffffffffll)
        return fail(QED_ERR_ARG, "qed_sorter_create: max_particles must be in [1, 2^32-1)");
    qed_sorter *s = new qed_sorter();
    s->max_particles = max_particles;
    s->hist_len = qed::radix_hist_len(max_particles);
    if (hipMalloc(&s->keys, sizeof(uint32_t) * 4 * max_particles) != hipSuccess ||
        hipMalloc(&s->hist, sizeof(uint32_t) * 2 * s->hist_len) != hipSuccess ||
        hipMalloc(&s->live, 64) != hipSuccess) {
        qed_sorter_free(s);
        return fail(QED_ERR_NOMEM, "qed_sorter_create: device allocation failed");
    }
    *out = s;
    return QED_OK;
}

void qed_sorter_free(qed_sorter *s) {
    if (!s) return;
    (void)hipFree(s->keys);
    (void)hipFree(s->hist);
    (void)hipFree(s->live);
    delete s;
}

qed_status qed_sort_by_cell(qed_sorter *so, qed_workspace *ws, qed_species *src, qed_species *dst,
                            const qed_field *grid, void *stream) {
    return qed_sort_by_cell_bands(so, ws, src, dst, grid, 1, stream);
}

qed_status qed_sort_by_cell_bands(qed_sorter *so, qed_workspace *ws, qed_species *src, qed_species *dst,
                                  const qed_field *grid, int32_t bands, void *stream) {
    if (bands != 1 && bands != 2 && bands != 4 && bands != 8)
        return fail(QED_ERR_ARG, "qed_sort_by_cell: bands must be 1, 2, 4 or 8");
    if (!so || !ws || !src || !dst || !grid) return fail(QED_ERR_ARG, "qed_sort_by_cell: null argument");
    if (grid->kind != QED_FIELD_YEE || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->dx > 0) ||
        !(grid->dy > 0) || !(grid->dz > 0))
        return fail(QED_ERR_ARG, "qed_sort_by_cell: needs a Yee grid geometry");
    const int64_t ncell = grid->nx * grid->ny * grid->nz;
    if (ncell >= (int64_t)0x7fffffff) return fail(QED_ERR_ARG, "qed_sort_by_cell: too many cells");
    qed::SortArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status st;
    if ((st = species_dev(src, false, "qed_sort_by_cell(src)", a.src))) return st;
    if ((st = species_dev(dst, false, "qed_sort_by_cell(dst)", a.dst))) return st;
    if (src->prec != dst->prec) return fail(QED_ERR_ARG, "qed_sort_by_cell: src and dst precisions differ");
    if (dst->capacity < src->capacity) return fail(QED_ERR_ARG, "qed_sort_by_cell: dst smaller than src");
    if (src->capacity > so->max_particles) return fail(QED_ERR_ARG, "qed_sort_by_cell: sorter too small");
    if ((src->chi == nullptr) != (dst->chi == nullptr)) return fail(QED_ERR_ARG, "qed_sort_by_cell: chi arrays differ");
    if (src->x == dst->x || src->tau == dst->tau || src->d_count == dst->d_count)
        return fail(QED_ERR_ARG, "qed_sort_by_cell: src and dst must be distinct buffers");
    // keys 0 .. (ncell + 1) bands - 1 (ncell: outside) < key_dead = 2^bits - 1
    const int64_t top = (ncell + 1) * bands - 1;
    if (top >= (int64_t)0xfffffffe) return fail(QED_ERR_ARG, "qed_sort_by_cell: too many cells for the bands");
    int bits = 1;
    while (((int64_t)1 << bits) - 1 <= top) ++bits;
    a.key_out = (uint32_t)ncell;
    a.key_dead = (uint32_t)(((uint64_t)1 << bits) - 1);
    a.bands = bands;
    a.x0 = grid->x0; a.y0 = grid->y0; a.z0 = grid->z0;
    a.inv_dx = 1.0 / grid->dx; a.inv_dy = 1.0 / grid->dy; a.inv_dz = 1.0 / grid->dz;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz;
    const int64_t m = so->max_particles;
    a.key0 = so->keys; a.key1 = so->keys + m; a.idx0 = so->keys + 2 * m; a.idx1 = so->keys + 3 * m;
    a.hist = so->hist; a.hoff = so->hist + so->hist_len;
    a.live = so->live;
    a.ws = ws->dev;
    HIP_TRY(qed::launch_sort(a, src->prec, bits, ws->n_cu, src->capacity, (hipStream_t)stream));
    return QED_OK;
}

// ------------------------------------------------------------------ merging --
qed_status qed_merger_create(int64_t max_particles, qed_merger **out) {
    if (!out) return fail(QED_ERR_ARG, "qed_merger_create: null out");
    *out = nullptr;
    if (max_particles < 1 || max_particles >= (int64_t)0xffffffffll)
        return fail(QED_ERR_ARG, "qed_merger_create: max_particles must be in [1, 2^32-1)");
    qed_merger *m = new qed_merger();
    m->max_particles = max_particles;
    m->hist_len = qed::radix_hist_len(max_particles);
    if (hipMalloc(&m->buf, sizeof(uint32_t) * (7 * max_particles + 2)) != hipSuccess ||
        hipMalloc(&m->hist, sizeof(uint32_t) * 2 * m->hist_len) != hipSuccess ||
        hipMalloc(&m->cnt, 64) != hipSuccess) {
        qed_merger_free(m);
        return fail(QED_ERR_NOMEM, "qed_merger_create: device allocation failed");
    }
    *out = m;
    return QED_OK;
}

void qed_merger_free(qed_merger *m) {
    if (!m) return;
    (void)hipFree(m->buf);
    (void)hipFree(m->hist);
    (void)hipFree(m->cnt);
    delete m;
}

static int bits_for(uint64_t v) {            // bits needed to hold the values 0..v
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

qed_status qed_merge(qed_merger *mg, qed_workspace *ws, const qed_merge_spec *sp, qed_species *src,
                     qed_species *dst, uint64_t seed, uint64_t *d_uid_next, void *stream) {
    if (!mg || !ws || !sp || !src || !dst || !d_uid_next) return fail(QED_ERR_ARG, "qed_merge: null argument");
    const int64_t lim = (int64_t)0x7fffffff;
    if (sp->nx < 1 || sp->ny < 1 || sp->nz < 1 || sp->nx > lim || sp->ny > lim || sp->nz > lim ||
        (double)sp->nx * (double)sp->ny * (double)sp->nz >= (double)(lim - 1))
        return fail(QED_ERR_ARG, "qed_merge: need 1 <= nx, ny, nz and nx ny nz < 2^31 - 2");
    if (!(sp->dx > 0) || !(sp->dy > 0) || !(sp->dz > 0) || !std::isfinite(sp->x0) || !std::isfinite(sp->y0) ||
        !std::isfinite(sp->z0))
        return fail(QED_ERR_ARG, "qed_merge: cell sizes must be > 0 and the origin finite");
    if (sp->n_octaves < 1 || sp->sub_bins < 1 || sp->sub_bins > 64 || (sp->sub_bins & (sp->sub_bins - 1)) ||
        sp->n_dir < 1 || sp->n_dir > 64 || sp->min_group < 2 || sp->octave_min < -1074 || sp->octave_min > 1023 ||
        (sp->massive != 0 && sp->massive != 1))
        return fail(QED_ERR_ARG, "qed_merge: bad energy or direction bins, min_group or massive flag");
    const double n_mbins = (double)sp->n_octaves * sp->sub_bins * 6.0 * sp->n_dir * sp->n_dir;
    if (n_mbins > 2147483648.0) return fail(QED_ERR_ARG, "qed_merge: more than 2^31 momentum bins");
    qed::MergeArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status st;
    if ((st = species_dev(src, false, "qed_merge(src)", a.src))) return st;
    if ((st = species_dev(dst, false, "qed_merge(dst)", a.dst))) return st;
    if (src->prec != dst->prec) return fail(QED_ERR_ARG, "qed_merge: src and dst precisions differ");
    if (dst->capacity < src->capacity) return fail(QED_ERR_ARG, "qed_merge: dst smaller than src");
    if (src->capacity > mg->max_particles) return fail(QED_ERR_ARG, "qed_merge: merger too small");
    if ((src->capacity + 4095) / 4096 > ws->max_tiles) return fail(QED_ERR_ARG, "qed_merge: workspace too small");
    if ((src->chi == nullptr) != (dst->chi == nullptr)) return fail(QED_ERR_ARG, "qed_merge: chi arrays differ");
    if (src->x == dst->x || src->tau == dst->tau || src->d_count == dst->d_count || src->uid == dst->uid)
        return fail(QED_ERR_ARG, "qed_merge: src and dst must be distinct buffers");
    const int64_t ncell = sp->nx * sp->ny * sp->nz;
    const int cbits = bits_for((uint64_t)ncell + 1);          // keys 0..ncell < key_dead = 2^cbits - 1
    a.key_out = (uint32_t)ncell;
    a.key_dead = (uint32_t)(((uint64_t)1 << cbits) - 1);
    const int mbits = bits_for((uint64_t)n_mbins - 1);
    a.x0 = sp->x0; a.y0 = sp->y0; a.z0 = sp->z0;
    a.inv_dx = 1.0 / sp->dx; a.inv_dy = 1.0 / sp->dy; a.inv_dz = 1.0 / sp->dz;
    a.nx = sp->nx; a.ny = sp->ny; a.nz = sp->nz;
    a.massive = sp->massive; a.octave_min = sp->octave_min; a.n_octaves = sp->n_octaves;
    a.sub_bins = sp->sub_bins; a.n_dir = sp->n_dir; a.min_group = sp->min_group;
    a.seed = seed;
    a.uid_next = d_uid_next;
    const int64_t m = mg->max_particles;
    a.key[0] = mg->buf; a.key[1] = mg->buf + m; a.idx[0] = mg->buf + 2 * m; a.idx[1] = mg->buf + 3 * m;
    a.mkey = mg->buf + 4 * m; a.g = mg->buf + 5 * m; a.o = mg->buf + 6 * m + 1;
    a.hist = mg->hist; a.hoff = mg->hist + mg->hist_len;
    a.cnt = mg->cnt;
    a.ws = ws->dev;
    HIP_TRY(qed::launch_merge(a, src->prec, (mbits + 7) / 8, (cbits + 7) / 8, ws->n_cu, (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_field_bound(const qed_field *f, int32_t block, float *bound, void *stream) {
    if (!f || f->kind != QED_FIELD_YEE || !f->grid || f->nx < 1 || f->ny < 1 || f->nz < 1)
        return fail(QED_ERR_ARG, "qed_field_bound: needs a Yee field with a grid");
    if (block < 1 || block > 64 || !bound) return fail(QED_ERR_ARG, "qed_field_bound: block in 1..64 and a table");
    HIP_TRY(qed::launch_field_bound(f->grid, f->nx, f->ny, f->nz, block, bound, (hipStream_t)stream));
    return QED_OK;
}

// ------------------------------------------------------------ PIC coupling --
static qed_status grid_geom(const qed_field *f, const char *who, qed::GridGeom &g) {
    if (!f || f->kind != QED_FIELD_YEE || f->nx < 1 || f->ny < 1 || f->nz < 1 || !(f->dx > 0) || !(f->dy > 0) ||
        !(f->dz > 0) || !std::isfinite(f->x0) || !std::isfinite(f->y0) || !std::isfinite(f->z0))
        return fail(QED_ERR_ARG, "%s: needs a Yee geometry (sizes >= 1, spacings > 0)", who);
    if ((double)f->nx * (double)f->ny * (double)f->nz > 9.0e15) return fail(QED_ERR_ARG, "%s: grid too large", who);
    g.nx = f->nx; g.ny = f->ny; g.nz = f->nz;
    g.x0 = f->x0; g.y0 = f->y0; g.z0 = f->z0;
    g.dx = f->dx; g.dy = f->dy; g.dz = f->dz;
    g.inv_dx = 1.0 / f->dx; g.inv_dy = 1.0 / f->dy; g.inv_dz = 1.0 / f->dz;
    return QED_OK;
}

static int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) return 256;
    return n;
}

qed_status qed_yee_advance(float *grid, const float *J, const qed_field *geometry, double dt, void *stream) {
    qed::GridGeom g;
    qed_status st;
    if ((st = grid_geom(geometry, "qed_yee_advance", g))) return st;
    if (!grid) return fail(QED_ERR_ARG, "qed_yee_advance: null grid");
    const double lim = 1.0 / std::sqrt(1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy) + 1.0 / (g.dz * g.dz));
    if (!(dt > 0.0) || !(dt < lim)) return fail(QED_ERR_ARG, "qed_yee_advance: dt must be in (0, %g)", lim);
    HIP_TRY(qed::launch_yee_advance(grid, J, g, dt, device_cus(), (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_deposit_current(const qed_species *s, const void *x_old, const void *y_old, const void *z_old,
                               const int64_t *d_first, double charge, double j_scale, double dt,
                               const qed_field *geometry, float *J, uint64_t *d_skipped, void *stream) {
    qed::DepositArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status st;
    if ((st = grid_geom(geometry, "qed_deposit_current", a.g))) return st;
    if ((st = species_dev(s, false, "qed_deposit_current", a.s))) return st;
    if (!J) return fail(QED_ERR_ARG, "qed_deposit_current: null J");
    if ((x_old == nullptr) != (y_old == nullptr) || (x_old == nullptr) != (z_old == nullptr))
        return fail(QED_ERR_ARG, "qed_deposit_current: give all three start arrays or none");
    if (!(dt > 0.0) || !std::isfinite(charge) || !std::isfinite(j_scale))
        return fail(QED_ERR_ARG, "qed_deposit_current: dt must be > 0, charge and j_scale finite");
    a.xo = x_old; a.yo = y_old; a.zo = z_old;
    a.d_first = d_first;
    a.q_scale = charge * j_scale;
    a.dt = dt;
    a.out = J;
    a.skipped = (unsigned long long *)d_skipped;
    HIP_TRY(qed::launch_deposit_current(a, s->prec, device_cus(), (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_deposit_charge(const qed_species *s, double charge, double j_scale, const qed_field *geometry,
                              float *rho, void *stream) {
    qed::DepositArgs a;
    std::memset(&a, 0, sizeof a);
    qed_status st;
    if ((st = grid_geom(geometry, "qed_deposit_charge", a.g))) return st;
    if ((st = species_dev(s, false, "qed_deposit_charge", a.s))) return st;
    if (!rho) return fail(QED_ERR_ARG, "qed_deposit_charge: null rho");
    if (!std::isfinite(charge) || !std::isfinite(j_scale))
        return fail(QED_ERR_ARG, "qed_deposit_charge: charge and j_scale must be finite");
    a.q_scale = charge * j_scale;
    a.out = rho;
    HIP_TRY(qed::launch_deposit_charge(a, s->prec, device_cus(), (hipStream_t)stream));
    return QED_OK;
}

qed_status qed_save_positions(const qed_species *s, void *x_old, void *y_old, void *z_old, void *stream) {
    qed::SpeciesDev d;
    qed_status st;
    if ((st = species_dev(s, false, "qed_save_positions", d))) return st;
    if (!x_old || !y_old || !z_old) return fail(QED_ERR_ARG, "qed_save_positions: null destination");
    HIP_TRY(qed::launch_save_positions(d, x_old, y_old, z_old, s->prec, device_cus(), (hipStream_t)stream));
    return QED_OK;
}

// ---------------------------------------------------------------- autotune --
qed_status qed_autotune_batched(const qed_tables *tab, qed_workspace *ws, const qed_units *u, double charge,
                                qed_species *lep, const qed_bunches *b, qed_species *ph_rec, const qed_step *st,
                                const qed_schedule *cand, int32_t n_cand, int32_t trial_steps,
                                const char *cache_path, qed_schedule *best, double *best_ms, void *stream) {
    if (!tab || !ws || !u || !lep || !b || !st || !cand || n_cand < 1 || trial_steps < 1 || !best)
        return fail(QED_ERR_ARG, "qed_autotune_batched: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    int64_t n = 0;
    HIP_TRY(hipMemcpy(&n, lep->d_count, sizeof n, hipMemcpyDeviceToHost));
    char key[256];
    snprintf(key, sizeof key, "n=%lld bunches=%d prec=%d rad=%d", (long long)n, b->n_bunches, lep->prec, st->rad_model);
    if (cache_path) {
        if (FILE *fp = std::fopen(cache_path, "r")) {
            char line[512];
            while (std::fgets(line, sizeof line, fp)) {
                qed_schedule c{};
                double ms = 0;
                char k2[256];
                if (std::sscanf(line, "%255[^|]| %d %d %d %d %lf", k2, &c.block, &c.items_per_thread, &c.blocks_per_cu,
                                &c.max_blocks, &ms) == 6 &&
                    std::strcmp(k2, key) == 0) {
                    std::fclose(fp);
                    *best = c;
                    if (best_ms) *best_ms = ms;
                    return QED_OK;
                }
            }
            std::fclose(fp);
        }
    }
    // scratch copy of the mutable lepton state, restored after each trial and
    // whatever happens; the workspace's status words and the recorded-photon
    // count are restored too, so trial appends leave no trace
    struct Scratch {
        void *saved = nullptr;
        double *t_energy = nullptr;
        int64_t *t_count = nullptr;
        uint64_t *t_uid = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Scratch() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            (void)hipFree(t_energy);
            (void)hipFree(t_count);
            (void)hipFree(t_uid);
            if (saved) (void)hipFree(saved);
        }
    } sc;
    const size_t es = lep->prec == QED_F64 ? 8 : 4;
    const size_t bytes = (size_t)n * (6 * es + 8 + 4);
    auto copy_state = [&](bool save) -> hipError_t {
        char *p = (char *)sc.saved;
        void *arr[6] = {lep->x, lep->y, lep->z, lep->ux, lep->uy, lep->uz};
        for (int k = 0; k < 6; ++k) {
            hipError_t e = save ? hipMemcpyAsync(p, arr[k], n * es, hipMemcpyDeviceToDevice, s)
                                : hipMemcpyAsync(arr[k], p, n * es, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
            p += n * es;
        }
        hipError_t e = save ? hipMemcpyAsync(p, lep->tau, n * 8, hipMemcpyDeviceToDevice, s)
                            : hipMemcpyAsync(lep->tau, p, n * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        p += n * 8;
        return save ? hipMemcpyAsync(p, lep->n_event, n * 4, hipMemcpyDeviceToDevice, s)
                    : hipMemcpyAsync(lep->n_event, p, n * 4, hipMemcpyDeviceToDevice, s);
    };
    int64_t rec_count0 = 0;
    unsigned long long status0[8];
    HIP_TRY(hipMemcpy(status0, ws->d_status, sizeof status0, hipMemcpyDeviceToHost));
    if (ph_rec) HIP_TRY(hipMemcpy(&rec_count0, ph_rec->d_count, sizeof rec_count0, hipMemcpyDeviceToHost));
    if (n > 0 && hipMalloc(&sc.saved, bytes) != hipSuccess) return fail(QED_ERR_NOMEM, "qed_autotune_batched: no scratch");
    HIP_TRY(hipMalloc(&sc.t_energy, sizeof(double) * QED_N_ENERGY));
    HIP_TRY(hipMalloc(&sc.t_count, sizeof(int64_t) * QED_N_COUNT));
    HIP_TRY(hipMalloc(&sc.t_uid, sizeof(uint64_t)));
    HIP_TRY(hipEventCreate(&sc.e0));
    HIP_TRY(hipEventCreate(&sc.e1));
    if (n > 0) HIP_TRY(copy_state(true));
    qed_tally tal{sc.t_energy, sc.t_count, 1};
    double best_t = 1e300;
    // the caller's state is first changed here: every path below restores it
    auto restore = [&]() -> qed_status {
        if (n > 0) HIP_TRY(copy_state(false));
        HIP_TRY(hipStreamSynchronize(s));
        if (ph_rec) HIP_TRY(hipMemcpy(ph_rec->d_count, &rec_count0, sizeof rec_count0, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(ws->d_status, status0, sizeof status0, hipMemcpyHostToDevice));
        return QED_OK;
    };
    auto trials = [&]() -> qed_status {
        for (int c = 0; c < n_cand; ++c) {
            const uint64_t big = 1ull << 62;
            HIP_TRY(hipMemcpy(sc.t_uid, &big, sizeof big, hipMemcpyHostToDevice));
            qed_step stc = *st;
            stc.d_step = nullptr;
            // one untimed warm-up step, then the timed trial
            qed_status rc = QED_OK;
            for (int k = 0; k <= trial_steps && rc == QED_OK; ++k) {
                if (k == 1) HIP_TRY(hipEventRecord(sc.e0, s));
                stc.t = st->t + k * st->dt;
                rc = qed_push_emit_batched(tab, ws, u, charge, lep, b, nullptr, ph_rec, &tal, &stc, sc.t_uid,
                                           &cand[c], stream);
            }
            HIP_TRY(hipEventRecord(sc.e1, s));
            HIP_TRY(hipEventSynchronize(sc.e1));
            float ms = 0;
            if (rc == QED_OK) {
                HIP_TRY(hipEventElapsedTime(&ms, sc.e0, sc.e1));
                if (ms < best_t) { best_t = ms; *best = cand[c]; }
            }                                       // an invalid candidate is skipped
            qed_status r = restore();
            if (r) return r;
        }
        return QED_OK;
    };
    qed_status rc = trials();
    if (rc) {
        const std::string msg = g_err;
        (void)restore();
        g_err = msg;
        return rc;
    }
    if (best_t >= 1e300) return fail(QED_ERR_ARG, "qed_autotune_batched: no valid candidate");
    if (best_ms) *best_ms = best_t / trial_steps;
    if (cache_path) {
        if (FILE *fp = std::fopen(cache_path, "a")) {
            std::fprintf(fp, "%s| %d %d %d %d %.6f\n", key, best->block, best->items_per_thread, best->blocks_per_cu,
                         best->max_blocks, best_t / trial_steps);
            std::fclose(fp);
        }
    }
    return QED_OK;
}

}  // extern "C"
