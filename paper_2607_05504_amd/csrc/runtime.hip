// Host side of the C ABI (include/sidm.h): context lifetime, scratch
// allocation sized once from the capacities, argument validation, and the
// stream-ordered launch of each step's kernels.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

#include "sidm_internal.h"

namespace {

// Allocation plan: every buffer the context owns, sized from the capacities.
struct Plan {
    struct Item { void **dst; size_t bytes; };
    static constexpr int kMax = 96;
    Item items[kMax];
    int n = 0;
    size_t total = 0;
    void add(void **dst, size_t bytes)
    {
        if (n >= kMax) abort();          // a buffer added without raising kMax
        bytes = (bytes + 255) & ~(size_t)255;
        items[n++] = Item{dst, bytes};
        total += bytes;
    }
};

// Candidates a step can list (accepted at the step start or at their turn):
// the configuration's max_accept, else a quarter of the active capacity, at
// least 65536.  The paper's criterion keeps every P(i|j) below C_SIDM; the
// benchmark workloads accept about 0.01 to 0.12 candidates per active
// particle.
int64_t acc_capacity(const sidm_config &cfg, int64_t cap_active)
{
    if (cfg.max_accept > 0) return cfg.max_accept;
    const int64_t floor_cap = (int64_t)1 << 16;
    const int64_t e = cap_active / 4;
    return e > floor_cap ? e : floor_cap;
}

// The phase buffer holds what only one call uses while it runs: the tree
// build's sort keys and values, then (over them) its 64-byte particle
// records; the neighbour search's leaf lists, counts, bounds and fallback
// list.  Offsets of each part, 256-byte aligned.
struct PhaseLayout {
    size_t key1, val0, val1, nl[2], fb[2], tb[2], total;
};
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
static PhaseLayout phase_layout(int64_t N, int64_t batch)
{
    PhaseLayout L;
    L.key1 = al256((size_t)N * 8);
    L.val0 = L.key1 + al256((size_t)N * 8);
    L.val1 = L.val0 + al256((size_t)N * 4);
    const size_t tree = L.val1 + al256((size_t)N * 4);
    const size_t rec = al256((size_t)N * 64);
    size_t o = al256((size_t)batch * SIDM_KNN_LMAX * 4);
    for (int q = 0; q < 2; ++q) {
        L.nl[q] = o; o += al256((size_t)batch * 4);
        L.fb[q] = o; o += al256((size_t)batch * 4);
        L.tb[q] = o; o += al256((size_t)batch * 8);
    }
    const size_t knn = o;
    L.total = tree > rec ? tree : rec;
    L.total = L.total > knn ? L.total : knn;
    return L;
}
static size_t phase_bytes(int64_t N, int64_t batch) { return phase_layout(N, batch).total; }

// the aliases into the phase buffer
static void carve_phase(sidm_ctx *c)
{
    const PhaseLayout L = phase_layout(c->cap_n, c->knn_batch);
    char *b = c->phase;
    c->key0 = (uint64_t *)b;
    c->key1 = (uint64_t *)(b + L.key1);
    c->val0 = (int32_t *)(b + L.val0);
    c->val1 = (int32_t *)(b + L.val1);
    c->rec = (double *)b;                  // written after the sort is done with the keys
    c->knn_list = (int32_t *)b;
    for (int q = 0; q < 2; ++q) {
        c->knn_nl[q] = (int32_t *)(b + L.nl[q]);
        c->knn_fb[q] = (int32_t *)(b + L.fb[q]);
        c->knn_tb[q] = (double *)(b + L.tb[q]);
    }
}

void make_plan(sidm_ctx *c, Plan &P)
{
    const int64_t N = c->cap_n, NA = c->cap_active;
    const int k = c->cfg.n_ngb;
    void **v;
#define ADD(field, count, type) v = (void **)&c->field; P.add(v, (size_t)(count) * sizeof(type))
    ADD(xs, N, double); ADD(ys, N, double); ADD(zs, N, double);
    ADD(vxs, N, double); ADD(vys, N, double); ADD(vzs, N, double); ADD(ms, N, double);
    ADD(ids, N, uint32_t); ADD(sts, N, uint8_t);
    ADD(perm, N, int32_t); ADD(inv, N, int32_t);
    const int64_t nsb = (N + SIDM_SORT_TILE - 1) / SIDM_SORT_TILE;
    ADD(hist, 256 * nsb, uint32_t);
    ADD(dtot, 6 * 256, uint32_t);
    ADD(bounds, 6, unsigned long long);
    ADD(nodes, tree_node_count(tree_levels(N)) * 6, double);
    ADD(sbox, tree_levels(N).cnt[0] * (SIDM_LEAF / SIDM_SUB) * 8, float);
    if (c->cfg.precision == SIDM_MIXED) {
        ADD(xo, N, float); ADD(yo, N, float); ADD(zo, N, float);
    }
    // neighbour-search batches of at most an eighth of the particles (at
    // least 65536 targets, at most SIDM_KNN_BATCH): their leaf lists share
    // the phase buffer below
    int64_t kb = N / 8 > ((int64_t)1 << 16) ? N / 8 : ((int64_t)1 << 16);
    kb = kb < SIDM_KNN_BATCH ? kb : SIDM_KNN_BATCH;
    c->knn_batch = NA < kb ? NA : kb;
    ADD(phase, phase_bytes(N, c->knn_batch), char);
    ADD(jsort, NA * (int64_t)k, int32_t);
    ADD(knn_fbn[0], 1, int32_t); ADD(knn_fbn[1], 1, int32_t);
    ADD(flag, N, int32_t);
    ADD(tlist, NA, int32_t); ADD(slot, NA, int32_t);
    ADD(blk, (N + SIDM_SCAN_TILE - 1) / SIDM_SCAN_TILE + 1, int32_t);
    ADD(nt_dev, 1, int32_t);
    const int64_t CA = acc_capacity(c->cfg, NA);
    // each listed candidate holds at most one record pair (the records of a
    // rewound turn are freed), so two records per listed candidate suffice
    const int64_t CR = 2 * CA;
    c->cap_acc = CA;
    c->cap_rec = CR;
    ADD(mem.i, CA, int32_t); ADD(mem.j, CA, int32_t); ADD(mem.cand, CA, int32_t);
    ADD(mem.u, CA, double); ADD(mem.W, CA, double); ADD(mem.dt, CA, double);
    ADD(mem.prio, CA, uint64_t); ADD(mem.idpair, CA, uint64_t); ADD(mem.rec, CA, int32_t);
    ADD(mmark, CA, int32_t);
    ADD(wl[0], CA, int32_t); ADD(wl[1], CA, int32_t);
    ADD(plist, 2 * CA, int32_t);
    ADD(trec.prio, CR, uint64_t); ADD(trec.idpair, CR, uint64_t);
    ADD(trec.vx, CR, double); ADD(trec.vy, CR, double); ADD(trec.vz, CR, double);
    ADD(trec.mem, CR, int32_t); ADD(trec.prev, CR, int32_t); ADD(trec.part, CR, int32_t);
    ADD(trec.info, CR, uint32_t);
    ADD(rfree, CR / 2, int32_t);
    ADD(head, N, int32_t);
    ADD(tmin, N, unsigned long long);
    ADD(dbits, (N + 31) / 32, uint32_t);
    ADD(bbits, bucket_words(N), uint32_t);
    if (k >= 4 && k <= SIDM_SUM_U && (k & (k - 1)) == 0)
        ADD(csum, (NA * (int64_t)k + SIDM_SUM_U - 1) / SIDM_SUM_U * SIDM_SUM_WORDS, int32_t);
    ADD(flist, 2 * SIDM_FLAG_CAP, int32_t);
    for (int b = 0; b < 2; ++b) {
        ADD(claim1[b], N, unsigned long long); ADD(claim2[b], N, unsigned long long);
    }
    ADD(acc_count, 16, int32_t);
    ADD(dstats, 1, DevStats);
    ADD(derr, 1, unsigned int);
    ADD(xt_w, SIDM_XSEC_TABLE_MAX, double); ADD(xt_s, SIDM_XSEC_TABLE_MAX, double);
    ADD(xt_lw, SIDM_XSEC_TABLE_MAX, double);
    ADD(adv_min, 1, unsigned long long);
    if (c->cfg.estimator == SIDM_EST_OVERLAP) {
        ADD(hs, N, double);
        ADD(hmax, tree_node_count(tree_levels(N)), double);
        ADD(gtab, (SIDM_OVERLAP_NA + 1) * (SIDM_OVERLAP_NR + 1), double);
    }
#undef ADD
}

void set_err(sidm_ctx *c, const char *fmt, ...)
{
    if (!c) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
}

// a stored -> physical factor: 0 (read as 1) or > 0 and finite
bool unit_factor_ok(double f) { return f == 0.0 || (f > 0.0 && f < 1e300); }

void normalize_units(sidm_config &cfg)
{
    if (cfg.len_to_phys == 0.0) cfg.len_to_phys = 1.0;
    if (cfg.vel_to_phys == 0.0) cfg.vel_to_phys = 1.0;
}

sidm_status check_config(const sidm_config *cfg)
{
    if (!cfg) return SIDM_E_INVAL;
    if (!unit_factor_ok(cfg->len_to_phys) || !unit_factor_ok(cfg->vel_to_phys))
        return SIDM_E_INVAL;
    if (cfg->n_ngb < 1 || cfg->n_ngb > 63) return SIDM_E_INVAL;
    if (cfg->max_accept < 0 || cfg->max_accept > ((int64_t)1 << 29)) return SIDM_E_INVAL;
    if (cfg->kernel != SIDM_KERNEL_CUBIC_SPLINE) return SIDM_E_INVAL;
    if (cfg->periodic && !(cfg->box > 0.0)) return SIDM_E_INVAL;
    if (cfg->xsec != SIDM_XSEC_CONST && cfg->xsec != SIDM_XSEC_YUKAWA &&
        cfg->xsec != SIDM_XSEC_TABLE)
        return SIDM_E_INVAL;
    if (cfg->xsec == SIDM_XSEC_TABLE) {
        if (cfg->xsec_n < 2 || cfg->xsec_n > SIDM_XSEC_TABLE_MAX || !cfg->xsec_w || !cfg->xsec_sigma)
            return SIDM_E_INVAL;
        for (int q = 0; q < cfg->xsec_n; ++q) {
            if (!(cfg->xsec_sigma[q] >= 0.0) || !(cfg->xsec_sigma[q] < 1e300)) return SIDM_E_INVAL;
            if (!(cfg->xsec_w[q] > 0.0) || !(cfg->xsec_w[q] < 1e300)) return SIDM_E_INVAL;
            if (q > 0 && !(cfg->xsec_w[q] > cfg->xsec_w[q - 1])) return SIDM_E_INVAL;
        }
    }
    if (cfg->xsec == SIDM_XSEC_YUKAWA && !(cfg->w0 > 0.0)) return SIDM_E_INVAL;
    if (cfg->model < SIDM_MODEL_ELASTIC || cfg->model > SIDM_MODEL_BEAM) return SIDM_E_INVAL;
    if (cfg->precision != SIDM_FP64 && cfg->precision != SIDM_MIXED) return SIDM_E_INVAL;
    if (!(cfg->c_sidm > 0.0)) return SIDM_E_INVAL;
    if (!(cfg->flag_band >= 0.0)) return SIDM_E_INVAL;
    if (cfg->estimator != SIDM_EST_ONE_SIDED && cfg->estimator != SIDM_EST_OVERLAP)
        return SIDM_E_INVAL;
    if (cfg->estimator == SIDM_EST_OVERLAP && cfg->precision != SIDM_FP64) return SIDM_E_INVAL;
    return SIDM_OK;
}

sidm_status hip_fail(sidm_ctx *c, hipError_t e, const char *what)
{
    set_err(c, "%s: %s", what, hipGetErrorString(e));
    return SIDM_E_DEVICE;
}

// Device errors latched by kernels, read without waiting (only when the host
// already synchronised); here we only translate the bits.
sidm_status status_from_bits(unsigned int bits)
{
    if (!bits) return SIDM_OK;
    if (bits & (DERR_OVERFLOW | DERR_NGB_OVERFLOW | DERR_HISTORY)) return SIDM_E_OVERFLOW;
    return SIDM_E_INVAL;
}

bool test_fail_alloc()
{
    const char *e = getenv("SIDM_TEST_FAIL_ALLOC");
    return e && e[0] == '1';
}

// rounds of the scattering step run as grid launches (the rest in one
// workgroup); tests lower it to exercise the one-workgroup tail
int test_device_rounds()
{
    const char *e = getenv("SIDM_TEST_DEVICE_ROUNDS");
    if (e && e[0] >= '0' && e[0] <= '9') return atoi(e);
    return 6;
}

// tests only: the row block summaries and the partner records also for the
// small steps they do not pay off on
int test_force_rows()
{
    const char *e = getenv("SIDM_TEST_FORCE_ROWS");
    return e && e[0] == '1';
}

}  // namespace

extern "C" {

const char *sidm_status_string(sidm_status s)
{
    switch (s) {
    case SIDM_OK: return "ok";
    case SIDM_E_INVAL: return "invalid argument";
    case SIDM_E_NOMEM: return "out of device memory";
    case SIDM_E_DEVICE: return "HIP runtime error";
    case SIDM_E_CAPACITY: return "capacity exceeded";
    case SIDM_E_OVERFLOW: return "accepted-candidate list or overlap row overflow";
    case SIDM_E_STATE: return "call out of order";
    }
    return "unknown status";
}

// the tabulated cross-section into the context (its host pointers are not
// kept: the caller's arrays may go away after sidm_create / sidm_reconfigure)
static hipError_t copy_table(sidm_ctx *c)
{
    if (c->cfg.xsec != SIDM_XSEC_TABLE) {
        c->cfg.xsec_w = c->cfg.xsec_sigma = nullptr;
        return hipSuccess;
    }
    const size_t b = (size_t)c->cfg.xsec_n * sizeof(double);
    double lw[SIDM_XSEC_TABLE_MAX];
    for (int q = 0; q < c->cfg.xsec_n; ++q) lw[q] = std::log(c->cfg.xsec_w[q]);
    hipError_t e = hipMemcpyAsync(c->xt_w, c->cfg.xsec_w, b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->xt_s, c->cfg.xsec_sigma, b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->xt_lw, lw, b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->cfg.xsec_w = c->cfg.xsec_sigma = nullptr;
    return e;
}

sidm_status sidm_footprint(const sidm_config *cfg, int64_t cap_n, int64_t cap_active, size_t *bytes)
{
    if (!bytes || check_config(cfg) != SIDM_OK) return SIDM_E_INVAL;
    if (cap_n < cfg->n_ngb + 2 || cap_active < 0 || cap_active > cap_n) return SIDM_E_INVAL;
    if (cap_active * (int64_t)cfg->n_ngb > (int64_t)INT32_MAX) return SIDM_E_CAPACITY;
    sidm_ctx tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.cfg = *cfg;
    tmp.cap_n = cap_n;
    tmp.cap_active = cap_active > 0 ? cap_active : 1;
    Plan P;
    make_plan(&tmp, P);
    *bytes = P.total;
    return SIDM_OK;
}

// the search's second stream and events (those that exist)
static void release_aux(sidm_ctx *c)
{
    if (c->knn_aux) {
        (void)hipStreamSynchronize(c->knn_aux);
        (void)hipStreamDestroy(c->knn_aux);
        c->knn_aux = nullptr;
    }
    for (int q = 0; q < 2; ++q)
        for (int e = 0; e < 2; ++e)
            if (c->knn_ev[q][e]) {
                (void)hipEventDestroy(c->knn_ev[q][e]);
                c->knn_ev[q][e] = nullptr;
            }
}

sidm_status sidm_create(const sidm_config *cfg, int64_t cap_n, int64_t cap_active, void *hip_stream,
                        sidm_ctx **out)
{
    if (!out) return SIDM_E_INVAL;
    *out = nullptr;
    if (check_config(cfg) != SIDM_OK) return SIDM_E_INVAL;
    if (cap_n < cfg->n_ngb + 2 || cap_n > ((int64_t)1 << 31) - 1 || cap_active < 1 ||
        cap_active > cap_n)
        return SIDM_E_INVAL;
    // a candidate's slot a * n_ngb + s is kept in 32 bits
    if (cap_active * (int64_t)cfg->n_ngb > (int64_t)INT32_MAX) return SIDM_E_CAPACITY;
    sidm_ctx *c = (sidm_ctx *)calloc(1, sizeof(sidm_ctx));
    if (!c) return SIDM_E_NOMEM;
    c->cfg = *cfg;
    normalize_units(c->cfg);
    c->cap_n = cap_n;
    c->cap_active = cap_active;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) { free(c); return SIDM_E_DEVICE; }
    Plan P;
    make_plan(c, P);
    char *base = nullptr;
    if (test_fail_alloc() || hipMalloc((void **)&base, P.total) != hipSuccess) {
        (void)hipGetLastError();
        free(c);
        return SIDM_E_NOMEM;
    }
    c->dev_base = base;
    size_t off = 0;
    for (int t = 0; t < P.n; ++t) {
        *P.items[t].dst = base + off;
        off += P.items[t].bytes;
    }
    carve_phase(c);
    c->jsort_ngb = nullptr;
    c->jsort_knn = 0;
    if (hipHostMalloc((void **)&c->hstats, sizeof(DevStats) + 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(base);
        free(c);
        return SIDM_E_NOMEM;
    }
    c->herr = (unsigned int *)((char *)c->hstats + sizeof(DevStats));
    // the search's second stream and its fork/join events
    bool ok = hipStreamCreateWithFlags(&c->knn_aux, hipStreamNonBlocking) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q)
        for (int e = 0; e < 2 && ok; ++e)
            ok = hipEventCreateWithFlags(&c->knn_ev[q][e], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        release_aux(c);
        (void)hipFree(base);
        (void)hipHostFree(c->hstats);
        free(c);
        return SIDM_E_DEVICE;
    }
    hipStream_t s = c->stream;
    // claims start cleared; error word and counters zero
    for (int b = 0; b < 2; ++b) {
        launch_fill_u64(c->claim1[b], ~0ull, cap_n, s);
        launch_fill_u64(c->claim2[b], ~0ull, cap_n, s);
    }
    launch_fill_i32((int32_t *)c->derr, 0, 1, s);
    launch_fill_i32(c->acc_count, 0, 16, s);
    // histories and replay marks start (and are left by every step) empty
    launch_fill_i32(c->head, -1, cap_n, s);
    launch_fill_u64(c->tmin, ~0ull, cap_n, s);
    launch_fill_i32(c->mmark, 0, c->cap_acc, s);
    launch_fill_i32((int32_t *)c->dbits, 0, (cap_n + 31) / 32, s);
    launch_fill_i32((int32_t *)c->bbits, 0, bucket_words(cap_n), s);
    c->dev_rounds = test_device_rounds();
    c->force_rows = test_force_rows();
    launch_fill_i32((int32_t *)c->dstats, 0, (int64_t)(sizeof(DevStats) / 4), s);
    hipError_t e = copy_table(c);
    if (e == hipSuccess && c->cfg.estimator == SIDM_EST_OVERLAP) e = launch_overlap_table(c);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(base);
        (void)hipHostFree(c->hstats);
        free(c);
        return SIDM_E_DEVICE;
    }
    c->err[0] = 0;
    *out = c;
    return SIDM_OK;
}

sidm_status sidm_timing_enable(sidm_ctx *c, int phases)
{
    if (!c) return SIDM_E_INVAL;
    if (phases & ~SIDM_TIMING_ALL) {
        set_err(c, "timing_enable: unknown phase bits 0x%x", (unsigned)phases);
        return SIDM_E_INVAL;
    }
    if (phases && !c->timing) {
        for (int p = 0; p < SIDM_PHASES; ++p)
            for (int r = 0; r < SIDM_TIMING_RING; ++r)
                for (int b = 0; b < 2; ++b)
                    if (!c->ev[p][r][b] && hipEventCreate(&c->ev[p][r][b]) != hipSuccess) {
                        set_err(c, "timing: hipEventCreate failed");
                        return SIDM_E_DEVICE;
                    }
    }
    for (int p = 0; p < SIDM_PHASES; ++p) c->ev_count[p] = 0;
    c->timing = phases;
    return SIDM_OK;
}

sidm_status sidm_timing_read(sidm_ctx *c, sidm_timing *out)
{
    if (!c || !out) return SIDM_E_INVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "timing_read");
    double v[SIDM_PHASES];
    int samples = 0;
    for (int p = 0; p < SIDM_PHASES; ++p) {
        double sum = 0.0;
        for (int r = 0; r < c->ev_count[p]; ++r) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, c->ev[p][r][0], c->ev[p][r][1]) == hipSuccess) sum += ms;
        }
        v[p] = c->ev_count[p] ? sum / c->ev_count[p] : 0.0;
        if (p == PH_KNN) samples = c->ev_count[p];
        c->ev_count[p] = 0;
    }
    out->samples = samples;
    out->tree_ms = v[PH_TREE];
    out->map_ms = v[PH_MAP];
    out->knn_ms = v[PH_KNN];
    out->eval_ms = v[PH_EVAL];
    out->resolve_ms = v[PH_RESOLVE];
    out->timestep_ms = v[PH_TIMESTEP];
    out->overlap_ms = v[PH_OVERLAP];
    return SIDM_OK;
}

sidm_status sidm_destroy(sidm_ctx *c)
{
    if (!c) return SIDM_E_INVAL;
    (void)hipStreamSynchronize(c->stream);
    release_aux(c);
    for (int p = 0; p < SIDM_PHASES; ++p)
        for (int r = 0; r < SIDM_TIMING_RING; ++r)
            for (int b = 0; b < 2; ++b)
                if (c->ev[p][r][b]) (void)hipEventDestroy(c->ev[p][r][b]);
    (void)hipFree(c->dev_base);
    (void)hipHostFree(c->hstats);
    free(c);
    return SIDM_OK;
}

sidm_status sidm_set_stream(sidm_ctx *c, void *hip_stream)
{
    if (!c) return SIDM_E_INVAL;
    c->stream = (hipStream_t)hip_stream;
    return SIDM_OK;
}

sidm_status sidm_reconfigure(sidm_ctx *c, const sidm_config *cfg)
{
    if (!c || !cfg) return SIDM_E_INVAL;
    if (check_config(cfg) != SIDM_OK) {
        set_err(c, "reconfigure: invalid configuration");
        return SIDM_E_INVAL;
    }
    if (cfg->n_ngb != c->cfg.n_ngb || cfg->precision != c->cfg.precision ||
        cfg->estimator != c->cfg.estimator || cfg->max_accept != c->cfg.max_accept) {
        set_err(c, "reconfigure: n_ngb, precision, estimator and max_accept fix the "
                   "context's layout");
        return SIDM_E_INVAL;
    }
    c->cfg = *cfg;
    normalize_units(c->cfg);
    c->tree_ok = 0;          // a new configuration needs a new snapshot
    c->map_valid = 0;
    c->jsort_ngb = nullptr;
    c->jsort_knn = 0;
    c->hs_valid = 0;
    hipError_t e = copy_table(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reconfigure");
    return SIDM_OK;
}

const char *sidm_last_error(const sidm_ctx *c)
{
    return c ? c->err : "null context";
}

static sidm_status check_particles(sidm_ctx *c, const sidm_particles *p, const char *who)
{
    if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->id) {
        set_err(c, "%s: NULL particle array", who);
        return SIDM_E_INVAL;
    }
    if (p->n < c->cfg.n_ngb + 2) {
        set_err(c, "%s: n=%lld < n_ngb+2", who, (long long)p->n);
        return SIDM_E_INVAL;
    }
    if (p->n > c->cap_n) {
        set_err(c, "%s: n=%lld above capacity %lld", who, (long long)p->n, (long long)c->cap_n);
        return SIDM_E_CAPACITY;
    }
    if (!p->mass && !(p->m_scalar > 0.0)) {
        set_err(c, "%s: no mass array and m_scalar <= 0", who);
        return SIDM_E_INVAL;
    }
    if ((c->cfg.model == SIDM_MODEL_TWO_STATE || c->cfg.model == SIDM_MODEL_BEAM) && !p->state) {
        set_err(c, "%s: the two-state and beam models need a state array", who);
        return SIDM_E_INVAL;
    }
    return SIDM_OK;
}

sidm_status sidm_refit_tree(sidm_ctx *c, const sidm_particles *p)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_particles(c, p, "refit_tree");
    if (st != SIDM_OK) return st;
    if (c->sorted_n != p->n) {
        set_err(c, "refit_tree: needs a sidm_build_tree of the same %lld particles first",
                (long long)p->n);
        return SIDM_E_STATE;
    }
    c->n = p->n;
    c->has_mass = p->mass != nullptr;
    c->m_scalar = p->m_scalar;
    c->jsort_ngb = nullptr;
    c->jsort_knn = 0;
    phase_begin(c, PH_TREE);
    hipError_t e = launch_refit_tree(c, p);
    phase_end(c, PH_TREE);
    c->map_valid = 0;
    c->hs_valid = 0;
    if (e != hipSuccess) return hip_fail(c, e, "refit_tree");
    c->tree_ok = 1;
    return SIDM_OK;
}

sidm_status sidm_build_tree(sidm_ctx *c, const sidm_particles *p)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_particles(c, p, "build_tree");
    if (st != SIDM_OK) return st;
    c->n = p->n;
    c->has_mass = p->mass != nullptr;
    c->m_scalar = p->m_scalar;
    c->jsort_ngb = nullptr;
    c->jsort_knn = 0;
    phase_begin(c, PH_TREE);
    hipError_t e = launch_build_tree(c, p);
    phase_end(c, PH_TREE);
    c->map_valid = 0;
    c->hs_valid = 0;
    if (e != hipSuccess) return hip_fail(c, e, "build_tree");
    c->tree_ok = 1;
    c->sorted_n = p->n;
    return SIDM_OK;
}

sidm_status sidm_tree_order(sidm_ctx *c, int32_t *order)
{
    if (!c) return SIDM_E_INVAL;
    if (!order) {
        set_err(c, "tree_order: NULL order");
        return SIDM_E_INVAL;
    }
    if (c->sorted_n <= 0) {
        set_err(c, "tree_order: sidm_build_tree has not been called");
        return SIDM_E_STATE;
    }
    hipError_t e = hipMemcpyAsync(order, c->perm, (size_t)c->sorted_n * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "tree_order");
    return SIDM_OK;
}

static sidm_status check_active(sidm_ctx *c, const int32_t *active, int64_t n_active, const char *who)
{
    if (!c->tree_ok) {
        set_err(c, "%s: sidm_build_tree has not been called", who);
        return SIDM_E_STATE;
    }
    if (n_active < 0) {
        set_err(c, "%s: bad active list", who);
        return SIDM_E_INVAL;
    }
    if (n_active > 0 && !active && !(c->map_valid && c->map_n == n_active)) {
        set_err(c, "%s: active == NULL needs an active set of %lld mapped by an earlier call "
                   "since the last tree build", who, (long long)n_active);
        return SIDM_E_STATE;
    }
    if (n_active > c->n) {
        set_err(c, "%s: n_active=%lld > n=%lld", who, (long long)n_active, (long long)c->n);
        return SIDM_E_INVAL;
    }
    if (n_active > c->cap_active) {
        set_err(c, "%s: n_active=%lld above capacity %lld", who, (long long)n_active,
                (long long)c->cap_active);
        return SIDM_E_CAPACITY;
    }
    return SIDM_OK;
}

// The active set in the tree's order: mapped from `active`, or (active ==
// NULL, checked by check_active) the mapping of the previous call reused.
// An empty set is always mapped, so the device-side target count is 0.
static hipError_t map_active(sidm_ctx *c, const int32_t *active, int64_t n_active)
{
    if (!active && n_active > 0) return hipSuccess;
    c->map_valid = 0;
    c->jsort_ngb = nullptr;
    c->jsort_knn = 0;
    hipError_t e = launch_map_active(c, active, n_active);
    if (e == hipSuccess) {
        c->map_valid = 1;
        c->map_n = n_active;
    }
    return e;
}

sidm_status sidm_find_ngb(sidm_ctx *c, const int32_t *active, int64_t n_active, int32_t *ngb, double *h)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_active(c, active, n_active, "find_ngb");
    if (st != SIDM_OK) return st;
    if (n_active > 0 && (!ngb || !h)) {
        set_err(c, "find_ngb: NULL output");
        return SIDM_E_INVAL;
    }
    if (n_active == 0) return SIDM_OK;
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess) e = launch_knn(c, n_active, ngb, h);
    // jsort now holds these rows in sorted indices, for this mapping
    c->jsort_ngb = nullptr;
    c->jsort_knn = e == hipSuccess && c->cfg.estimator == SIDM_EST_ONE_SIDED;
    if (e != hipSuccess) return hip_fail(c, e, "find_ngb");
    return SIDM_OK;
}

sidm_status sidm_scatter_step(sidm_ctx *c, sidm_particles *p, const int32_t *active, int64_t n_active,
                              const int32_t *ngb, const double *h, const double *dt, uint64_t seed,
                              uint32_t step, uint32_t *cand_info)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_active(c, active, n_active, "scatter_step");
    if (st != SIDM_OK) return st;
    if (!p || p->n != c->n || !p->vx || !p->vy || !p->vz) {
        set_err(c, "scatter_step: particles do not match the tree snapshot");
        return SIDM_E_INVAL;
    }
    if (c->cfg.model == SIDM_MODEL_TWO_STATE && !p->state) {
        set_err(c, "scatter_step: two-state model needs a state array");
        return SIDM_E_INVAL;
    }
    if (n_active > 0 && (!ngb || !h || !dt)) {
        set_err(c, "scatter_step: NULL ngb/h/dt");
        return SIDM_E_INVAL;
    }
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess) e = launch_scatter(c, p, n_active, ngb, h, dt, seed, step, cand_info);
    if (e != hipSuccess) return hip_fail(c, e, "scatter_step");
    return SIDM_OK;
}

sidm_status sidm_pair_timestep(sidm_ctx *c, const int32_t *active, int64_t n_active, const int32_t *ngb,
                               const double *h, double *dt_sidm)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_active(c, active, n_active, "pair_timestep");
    if (st != SIDM_OK) return st;
    if (n_active > 0 && (!ngb || !h || !dt_sidm)) {
        set_err(c, "pair_timestep: NULL ngb/h/dt_sidm");
        return SIDM_E_INVAL;
    }
    if (n_active == 0) return SIDM_OK;
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess) e = launch_timestep(c, n_active, ngb, h, dt_sidm);
    if (e != hipSuccess) return hip_fail(c, e, "pair_timestep");
    return SIDM_OK;
}

static sidm_status check_overlap(sidm_ctx *c, const double *h_all, const int32_t *active,
                                 int64_t n_active, int32_t max_ngb, const void *ngb,
                                 const int32_t *count, const char *who)
{
    if (c->cfg.estimator != SIDM_EST_OVERLAP) {
        set_err(c, "%s: the context was created without estimator SIDM_EST_OVERLAP", who);
        return SIDM_E_STATE;
    }
    sidm_status st = check_active(c, active, n_active, who);
    if (st != SIDM_OK) return st;
    if (max_ngb < 1) {
        set_err(c, "%s: max_ngb=%d < 1", who, (int)max_ngb);
        return SIDM_E_INVAL;
    }
    if (n_active > 0 && (!h_all || !ngb || !count)) {
        set_err(c, "%s: NULL h_all/ngb/count", who);
        return SIDM_E_INVAL;
    }
    if (n_active * (int64_t)max_ngb > (int64_t)INT32_MAX) {
        set_err(c, "%s: n_active * max_ngb = %lld does not fit the 32-bit slot index", who,
                (long long)(n_active * (int64_t)max_ngb));
        return SIDM_E_CAPACITY;
    }
    return SIDM_OK;
}

sidm_status sidm_find_overlap(sidm_ctx *c, double *h_all, const int32_t *active,
                              const double *h_active, int64_t n_active, int32_t max_ngb,
                              int32_t *ngb, int32_t *count)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_overlap(c, h_all, active, n_active, max_ngb, ngb, count, "find_overlap");
    if (st != SIDM_OK) return st;
    if (n_active == 0) return SIDM_OK;
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess)
        e = launch_find_overlap(c, h_all, h_active, n_active, max_ngb, ngb, count);
    if (e != hipSuccess) return hip_fail(c, e, "find_overlap");
    return SIDM_OK;
}

sidm_status sidm_scatter_overlap(sidm_ctx *c, sidm_particles *p, const double *h_all,
                                 const int32_t *active, int64_t n_active, int32_t max_ngb,
                                 const int32_t *ngb, const int32_t *count, const double *dt,
                                 uint64_t seed, uint32_t step, uint32_t *cand_info)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_overlap(c, h_all, active, n_active, max_ngb, ngb, count,
                                   "scatter_overlap");
    if (st != SIDM_OK) return st;
    if (!p || p->n != c->n || !p->vx || !p->vy || !p->vz) {
        set_err(c, "scatter_overlap: particles do not match the tree snapshot");
        return SIDM_E_INVAL;
    }
    if ((c->cfg.model == SIDM_MODEL_TWO_STATE || c->cfg.model == SIDM_MODEL_BEAM) && !p->state) {
        set_err(c, "scatter_overlap: the two-state and beam models need a state array");
        return SIDM_E_INVAL;
    }
    if (n_active > 0 && !dt) {
        set_err(c, "scatter_overlap: NULL dt");
        return SIDM_E_INVAL;
    }
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess && n_active > 0 && !(c->hs_valid && c->hs_src == h_all))
        e = launch_gather_h(c, h_all);
    if (e == hipSuccess)
        e = launch_scatter_overlap(c, p, n_active, max_ngb, ngb, count, dt, seed, step,
                                   cand_info);
    if (e != hipSuccess) return hip_fail(c, e, "scatter_overlap");
    return SIDM_OK;
}

sidm_status sidm_pair_timestep_overlap(sidm_ctx *c, const double *h_all, const int32_t *active,
                                       int64_t n_active, int32_t max_ngb, const int32_t *ngb,
                                       const int32_t *count, double *dt_sidm)
{
    if (!c) return SIDM_E_INVAL;
    sidm_status st = check_overlap(c, h_all, active, n_active, max_ngb, ngb, count,
                                   "pair_timestep_overlap");
    if (st != SIDM_OK) return st;
    if (n_active > 0 && !dt_sidm) {
        set_err(c, "pair_timestep_overlap: NULL dt_sidm");
        return SIDM_E_INVAL;
    }
    if (n_active == 0) return SIDM_OK;
    hipError_t e = map_active(c, active, n_active);
    if (e == hipSuccess && !(c->hs_valid && c->hs_src == h_all)) e = launch_gather_h(c, h_all);
    if (e == hipSuccess) e = launch_timestep_overlap(c, n_active, max_ngb, ngb, count, dt_sidm);
    if (e != hipSuccess) return hip_fail(c, e, "pair_timestep_overlap");
    return SIDM_OK;
}

sidm_status sidm_overlap_table(sidm_ctx *c, double *host_out)
{
    if (!c || !host_out) return SIDM_E_INVAL;
    if (c->cfg.estimator != SIDM_EST_OVERLAP) {
        set_err(c, "overlap_table: the context was created without estimator SIDM_EST_OVERLAP");
        return SIDM_E_STATE;
    }
    const size_t b = (size_t)(SIDM_OVERLAP_NA + 1) * (SIDM_OVERLAP_NR + 1) * sizeof(double);
    hipError_t e = hipMemcpyAsync(host_out, c->gtab, b, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "overlap_table");
    return SIDM_OK;
}

sidm_status sidm_advance_hernquist(sidm_ctx *c, double *x, double *y, double *z, double *vx,
                                   double *vy, double *vz, int64_t n, const double *dt_sidm,
                                   int64_t n_active, double dt_cap, double gm, double a,
                                   double *dt_next, double *dt_step)
{
    if (!c) return SIDM_E_INVAL;
    if (n < 0 || n > c->cap_n || n_active < 0 || n_active > n) {
        set_err(c, "advance_hernquist: n=%lld n_active=%lld cap_n=%lld", (long long)n,
                (long long)n_active, (long long)c->cap_n);
        return SIDM_E_INVAL;
    }
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz)) {
        set_err(c, "advance_hernquist: NULL particle array");
        return SIDM_E_INVAL;
    }
    if (n_active > 0 && !dt_sidm) {
        set_err(c, "advance_hernquist: NULL dt_sidm");
        return SIDM_E_INVAL;
    }
    if (!(dt_cap > 0.0) || !(dt_cap < 1e300) || !(gm >= 0.0) || !(a > 0.0)) {
        set_err(c, "advance_hernquist: need dt_cap > 0, gm >= 0, a > 0");
        return SIDM_E_INVAL;
    }
    if (n == 0) return SIDM_OK;
    hipError_t e = launch_advance(c, x, y, z, vx, vy, vz, n, dt_sidm, n_active, dt_cap, gm, a,
                                  dt_next, dt_step);
    if (e != hipSuccess) return hip_fail(c, e, "advance_hernquist");
    return SIDM_OK;
}

sidm_status sidm_drift(sidm_ctx *c, double *x, double *y, double *z, const double *vx,
                       const double *vy, const double *vz, int64_t n, double dt)
{
    if (!c) return SIDM_E_INVAL;
    if (n < 0 || n > c->cap_n) {
        set_err(c, "drift: n=%lld cap_n=%lld", (long long)n, (long long)c->cap_n);
        return SIDM_E_INVAL;
    }
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz)) {
        set_err(c, "drift: NULL particle array");
        return SIDM_E_INVAL;
    }
    if (!(dt >= 0.0) || !(dt < 1e300)) {
        set_err(c, "drift: need a finite dt >= 0");
        return SIDM_E_INVAL;
    }
    if (n == 0) return SIDM_OK;
    hipError_t e = launch_drift(c, x, y, z, vx, vy, vz, n, dt);
    if (e != hipSuccess) return hip_fail(c, e, "drift");
    return SIDM_OK;
}

sidm_status sidm_sync(sidm_ctx *c, sidm_stats *out)
{
    if (!c) return SIDM_E_INVAL;
    hipError_t e = hipMemcpyAsync(c->hstats, c->dstats, sizeof(DevStats), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->herr, c->derr, sizeof(unsigned int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sync");
    unsigned int bits = *c->herr;
    sidm_status st = status_from_bits(bits);
    if (out) {
        const DevStats &d = *c->hstats;
        out->n_cand = (int64_t)d.n_cand;
        out->n_accept0 = (int64_t)d.n_accept0;
        out->n_events = (int64_t)d.n_events;
        out->n_flagged = (int64_t)d.n_flagged;
        out->n_p_ge_1 = (int64_t)d.n_p_ge_1;
        out->n_recheck = (int64_t)d.n_recheck;
        out->n_passes = (int32_t)d.n_passes;
        out->n_rounds = (int32_t)d.n_rounds;
        out->error = (int32_t)st;
        unsigned long long mb = d.max_p_bits;
        double mp;
        memcpy(&mp, &mb, sizeof mp);
        out->max_p = mp;
    }
    if (bits) {
        set_err(c, "device error bits 0x%x (%s%s%s%s%s%s%s%s)", bits,
                (bits & DERR_INDEX) ? "index " : "",
                (bits & DERR_DUPLICATE) ? "duplicate-active " : "",
                (bits & DERR_OVERFLOW) ? "accepted-overflow " : "",
                (bits & DERR_COUNT) ? "too-few-neighbours " : "",
                (bits & DERR_STALL) ? "stalled-resolution " : "",
                (bits & DERR_NGB_OVERFLOW) ? "overlap-row-overflow " : "",
                (bits & DERR_BAD_H) ? "bad-smoothing-length " : "",
                (bits & DERR_HISTORY) ? "history-overflow " : "");
        launch_fill_i32((int32_t *)c->derr, 0, 1, c->stream);
        (void)hipStreamSynchronize(c->stream);
    }
    return st;
}

}  // extern "C"
