/*
 * sidm.h -- C ABI of the MI355X (gfx950) SIDM scattering step.
 *
 * The library performs the Monte-Carlo self-interacting dark matter
 * scattering step of Zier et al., "A Novel Implementation of Self-Interacting
 * Dark Matter in AREPO" (arXiv 2607.05504) on one GPU:
 *
 *   sidm_build_tree     spatial sort + bucket tree of the DM particles
 *                       (the dedicated DM-only neighbour tree of sec. 4.3)
 *   sidm_find_ngb       N_ngb nearest neighbours and smoothing length of every
 *                       active particle (sec. 4.2, 4.5)
 *   sidm_scatter_step   pair probabilities P(i|j) (Eqs. rate, oneSided,
 *                       probabilityScatter), random draws, conflict resolution
 *                       and momentum/energy-conserving kicks (sec. 4.1, 4.5)
 *   sidm_pair_timestep  per-pair timestep bound (Eq. sidm_timestep, sec. 4.4)
 *
 * and, for the served form (many independent haloes stepped concurrently,
 * one context and stream each), sidm_advance_hernquist: the global step
 * length from the per-pair bounds and a leapfrog step in a fixed halo
 * potential between scattering steps.
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers on the context's device, owned
 *     by the caller (for example torch tensors' data_ptr()).  The library
 *     owns only the scratch it allocates in sidm_create; no call after
 *     sidm_create allocates device memory.
 *   - Every call is asynchronous and ordered on the context's HIP stream.
 *     (sidm_find_ngb runs part of its work on a second stream the context
 *     creates, of default priority, forked from and joined back to the
 *     context's stream with events inside the call, so the ordering seen by
 *     the caller is the same.)
 *     Errors found on the host (bad sizes, NULL pointers, capacity) are
 *     returned before anything is enqueued and leave every array untouched.
 *     Errors found by a kernel (an index out of range, a duplicate active
 *     entry, an overflowing accepted list) are latched in the context and
 *     returned by sidm_sync (and by the next call that checks them).
 *   - Indices in `active` and `ngb` are in the caller's particle order.
 *   - Every call that takes `active` first maps the active set into the
 *     tree's order.  Given active == NULL (and n_active > 0) a call reuses the
 *     mapping of the previous call on the context instead, which must have
 *     had the same n_active, with no sidm_build_tree, sidm_refit_tree or
 *     sidm_reconfigure since (SIDM_E_STATE otherwise): for example
 *     sidm_scatter_step and sidm_pair_timestep after sidm_find_ngb of the
 *     same step.
 *   - A context is not thread-safe.  Distinct contexts are independent and
 *     may run concurrently on different streams.
 *
 * Semantics fixed by this library where the paper leaves them open:
 *   - N(i) is the set of the n_ngb particles j != i with the smallest
 *     (r_ij^2, id_j), inactive particles included; h_i is the distance of the
 *     (n_ngb+1)-th, so every neighbour lies inside the kernel support (the
 *     paper iterates h to 32 +- 5 neighbours).  Distances use the minimum
 *     image in a periodic box:  d = x_j - x_i;  d >= L/2 -> d - L;
 *     d < -L/2 -> d + L;  r^2 = (dx*dx + dy*dy) + dz*dz.
 *   - P(i|j) = ((((1/2 m_j) sigma(w)/m) w) W(r_ij, h_i)) dt_i with
 *     w = |v_i - v_j|, the cubic-spline W of sec. 4.2.
 *   - Random numbers: Philox4x32-10 keyed on `seed`, counter (min id,
 *     max id, step, purpose); purpose 0 decides, 1/3 give the direction for
 *     the lower/higher-ID target, 2 gives the priority.  Of a draw's words,
 *     (x0, x1) serve the lower-ID target and (x2, x3) the higher-ID target;
 *     u = (word >> 11) * 2^-53.
 *   - Every directed candidate (i|j) takes exactly one turn, in increasing
 *     (priority, id_i, id_j) with the priority word of the pair's draw; at
 *     its turn P is computed with the velocities (and states) of that moment
 *     and the candidate scatters iff u < P (sec. 4.5: a pair evaluated after
 *     a kick of one of its particles sees the updated state).  The result is
 *     exactly that serial order; the device gets it in parallel (passes in
 *     which every particle scatters with at most one partner, and rounds
 *     that check every candidate at its turn against the particles'
 *     histories within the step, see scatter.hip).
 */
#ifndef SIDM_H
#define SIDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIDM_OK = 0,
    SIDM_E_INVAL = -1,     /* invalid argument (host) or invalid index/duplicate (device) */
    SIDM_E_NOMEM = -2,     /* device allocation failed in sidm_create                  */
    SIDM_E_DEVICE = -3,    /* HIP runtime error                                        */
    SIDM_E_CAPACITY = -4,  /* n or n_active above the context's capacity               */
    SIDM_E_OVERFLOW = -5,  /* accepted-candidate list or an overlap row overflowed     */
    SIDM_E_STATE = -6      /* call out of order (e.g. find_ngb before build_tree)      */
} sidm_status;

enum { SIDM_KERNEL_CUBIC_SPLINE = 0 };
enum { SIDM_XSEC_CONST = 0, SIDM_XSEC_YUKAWA = 1, SIDM_XSEC_TABLE = 2 };
#define SIDM_XSEC_TABLE_MAX 256   /* nodes of a tabulated cross-section */
enum { SIDM_MODEL_ELASTIC = 0, SIDM_MODEL_EPS = 1, SIDM_MODEL_TWO_STATE = 2, SIDM_MODEL_BEAM = 3 };
enum { SIDM_FP64 = 0, SIDM_MIXED = 1 };
/* scattering-rate estimator (sec. 4.2): the fiducial one-sided kernel, or the
 * kernel overlap of Eq. kernelOverlap (the *_overlap calls) */
enum { SIDM_EST_ONE_SIDED = 0, SIDM_EST_OVERLAP = 1 };
/* the overlap estimator's table of ghat(alpha, rho): alpha = a / (2 NA),
 * a = 0..NA; rho = b / NR, b = 0..NR; stored alpha-major */
#define SIDM_OVERLAP_NA 64
#define SIDM_OVERLAP_NR 256

/* per-candidate info word (optional output of sidm_scatter_step) */
#define SIDM_CAND_ACCEPT0 1u   /* u < P with the step-start velocities (diagnostic) */
#define SIDM_CAND_SCATTER 2u   /* kicked at its turn                                */
#define SIDM_CAND_FLAGGED 4u   /* |P - u| < flag_band at its turn                   */
/* bits 8..31: a kick's depth, 1 + the larger depth of the last earlier kicks
 * of its two particles (0 if none): the pass in which a parallel matching of
 * the kicks in turn order applies it.  0 for a candidate that did not kick. */

typedef struct {
    int32_t n_ngb;        /* neighbours per target, 1..63 (paper: 32)                    */
    int32_t kernel;       /* SIDM_KERNEL_CUBIC_SPLINE                                     */
    int32_t periodic;     /* 1: periodic cube [0, box)^3 with minimum image; 0: open      */
    int32_t xsec;         /* SIDM_XSEC_CONST: sigma/m = sigma0;
                             SIDM_XSEC_YUKAWA: sigma0 / (1 + (w/w0)^2)^2;
                             SIDM_XSEC_TABLE: the table below                              */
    int32_t model;        /* SIDM_MODEL_ELASTIC (eps = 1), SIDM_MODEL_EPS (constant eps),
                             SIDM_MODEL_TWO_STATE (ground/excited, gap delta per unit mass),
                             SIDM_MODEL_BEAM (the fixed-target beam test of sec. 5.1:
                             state 1 = beam, 0 = target; only beam-target pairs scatter,
                             elastically, and the target does not recoil) */
    int32_t precision;    /* SIDM_FP64, or SIDM_MIXED (FP32 probabilities with an FP64
                             recheck inside band_p; the neighbour search is the exact
                             FP64 one in both forms; kicks stay FP64)                     */
    double box;           /* periodic box side L                                          */
    double sigma0, w0;    /* cross-section parameters                                     */
    double eps, delta;    /* constant eps; two-state energy gap per unit mass             */
    double c_sidm;        /* timestep coefficient (paper: 0.1)                            */
    double flag_band;     /* evaluations with |P - u| < flag_band are flagged (1e-9)      */
    double band_r2;       /* kept for layout; no effect (the search is FP64 in both forms)*/
    double band_p;        /* mixed form: relative |P - u| band rechecked in FP64          */
    /* SIDM_XSEC_TABLE (a tabulated sigma(w)/m of the pair's relative speed,
     * sec. 4.2, as the velocity-dependent models of sec. 6 are given):
     * xsec_n nodes (2..SIDM_XSEC_TABLE_MAX) at strictly increasing speeds
     * xsec_w > 0 with values xsec_sigma >= 0; between the nodes w_k <= w <
     * w_k+1 sigma is linear in ln w (the interpolation in log velocity the
     * paper uses), sigma_k + (ln w - ln w_k) / (ln w_k+1 - ln w_k)
     * (sigma_k+1 - sigma_k); outside the range it is the end value.  HOST pointers, copied into the context by sidm_create
     * and sidm_reconfigure (not read afterwards); ignored for other xsec. */
    int32_t xsec_n;
    const double *xsec_w;
    const double *xsec_sigma;
    /* SIDM_EST_ONE_SIDED (0; sidm_scatter_step's g_ij = W(r_ij, h_i)) or
     * SIDM_EST_OVERLAP, which also reserves what the *_overlap calls need (a
     * Morton-ordered copy of every particle's h, the largest h of every tree
     * node, the ghat table; 8 bytes a particle more) and requires
     * precision SIDM_FP64. */
    int32_t estimator;
    /* Stored -> physical units (sec. 4.2: cosmological runs store comoving
     * coordinates and velocities and evaluate the pair rate in physical
     * units).  Separations and smoothing lengths are multiplied by
     * len_to_phys (the scale factor a for comoving positions) and relative
     * speeds by vel_to_phys (the factor of the caller's velocity variable)
     * wherever W, g_ij, sigma(w), P, the two-state energy balance and the
     * timestep use them; the search and the kick stay in stored units (the
     * kick changes no speed but through eps).  dt is taken as given.  0 (or
     * 1) for physical storage; otherwise > 0 and finite (SIDM_E_INVAL). */
    double len_to_phys;
    double vel_to_phys;
    /* Largest number of candidates one scattering step can list for the
     * ordered replay of turns: those accepted with the step-start velocities
     * plus those found to accept only at their turn.  A step that needs
     * more latches SIDM_E_OVERFLOW (sidm_sync).  0: a quarter of
     * cap_active, at least 65536.  Device memory grows by about 190 bytes
     * per listed candidate.  0 .. 2^29. */
    int64_t max_accept;
} sidm_config;

typedef struct {
    const double *x, *y, *z;     /* positions [n]                                        */
    double *vx, *vy, *vz;        /* velocities [n]; updated by sidm_scatter_step         */
    const double *mass;          /* per-particle mass [n], or NULL to use m_scalar        */
    double m_scalar;
    const uint32_t *id;          /* unique particle IDs [n] (tie-break and RNG key)      */
    uint8_t *state;              /* internal state bit [n] (two-state model), else NULL   */
    int64_t n;
} sidm_particles;

typedef struct {
    int64_t n_cand;       /* candidates evaluated at step start (n_active * n_ngb)       */
    int64_t n_accept0;    /* accepted at step start                                      */
    int64_t n_events;     /* kicks applied                                               */
    int64_t n_flagged;    /* turns with |P - u| < flag_band                              */
    int64_t n_p_ge_1;     /* step-start evaluations with P >= 1 (always accepted)        */
    int64_t n_recheck;    /* mixed form: evaluations redone in FP64                      */
    int32_t n_passes;     /* largest kick depth (see SIDM_CAND_* above)                  */
    int32_t error;        /* latched sidm_status of the device, 0 if none                */
    double max_p;         /* largest step-start P                                        */
    int32_t n_rounds;     /* checks of the turn order run (1: the candidates accepted at
                             the step start were all that acted)                          */
    int32_t pad;
} sidm_stats;

typedef struct sidm_ctx sidm_ctx;

/* Device bytes sidm_create would allocate for these capacities (the serving
 * layer admits work against an HBM budget with it).  No device work. */
sidm_status sidm_footprint(const sidm_config *cfg, int64_t cap_n, int64_t cap_active,
                           size_t *bytes);

/* Create a context on the current HIP device with capacity for cap_n
 * particles and cap_active active particles; `hip_stream` (hipStream_t, may be
 * NULL for the default stream) orders all its work.  The context also creates
 * one stream of its own (default priority) and four events for the neighbour
 * search; sidm_destroy releases them.  *out receives the context, or NULL on
 * error (SIDM_E_NOMEM, or SIDM_E_DEVICE if the stream or events cannot be
 * created). */
sidm_status sidm_create(const sidm_config *cfg, int64_t cap_n, int64_t cap_active,
                        void *hip_stream, sidm_ctx **out);
sidm_status sidm_destroy(sidm_ctx *ctx);
sidm_status sidm_set_stream(sidm_ctx *ctx, void *hip_stream);
/* Replace the context's configuration (for example sigma0 of the next halo a
 * pooled context serves).  n_ngb, precision, estimator and max_accept fix the
 * context's memory layout and must not change (SIDM_E_INVAL otherwise, context unchanged).  The next
 * step needs a new sidm_build_tree.  Host-side only; call it between steps
 * (work already enqueued keeps the old values). */
sidm_status sidm_reconfigure(sidm_ctx *ctx, const sidm_config *cfg);

/* Last error message of the context (host-side text), "" if none. */
const char *sidm_last_error(const sidm_ctx *ctx);
const char *sidm_status_string(sidm_status s);

/* Snapshot and spatially sort the particles (all of them, active or not:
 * inactive particles are neighbours too).  The calls that follow read
 * positions and velocities from this snapshot, and sidm_scatter_step keeps it
 * in step with the velocity/state updates it writes back to the caller's
 * arrays.  The caller must not change x, v or state between sidm_build_tree
 * and the last call of the step.  Requires n_ngb + 2 <= n <= cap_n. */
sidm_status sidm_build_tree(sidm_ctx *ctx, const sidm_particles *p);

/* Tree reuse across steps: the snapshot and every box are rebuilt from the
 * particles' current positions and velocities, in the Morton order of the
 * last sidm_build_tree (no sort).  Results stay exact; the search slows as
 * the particles move away from that order.  Requires a sidm_build_tree of the
 * same number of particles earlier on this context (SIDM_E_STATE otherwise);
 * other requirements as for sidm_build_tree. */
sidm_status sidm_refit_tree(sidm_ctx *ctx, const sidm_particles *p);

/* The tree's particle order (sec. 4.3: particles sorted along the
 * space-filling curve): order[s] = caller index of the particle at sorted
 * position s, for the n particles of the last sidm_build_tree -- ascending
 * 48-bit Morton keys of the positions quantised to 16 bits an axis over the
 * bounding box (over [0, box) when periodic), equal keys in caller order.
 * order: caller-owned device array of n int32.  Asynchronous on the
 * context's stream; SIDM_E_STATE before the first sidm_build_tree.  For
 * callers that keep their particles in tree order, and for checking the sort. */
sidm_status sidm_tree_order(sidm_ctx *ctx, int32_t *order);

/* For every active particle a (0 <= a < n_active, active[a] a particle
 * index, no duplicates): ngb[a*n_ngb + s] = its s-th nearest neighbour
 * (ascending (r^2, id)), h[a] = distance of the (n_ngb+1)-th (sec. 4.2:
 * a fixed neighbour number sets h).  Exact in both precision forms.  The
 * search runs in batches; with more than one batch the root walks of a
 * batch's hard targets run on the context's second stream while the next
 * batch is searched, and the call joins them back before it returns. */
sidm_status sidm_find_ngb(sidm_ctx *ctx, const int32_t *active, int64_t n_active,
                          int32_t *ngb, double *h);

/* One scattering step of the active particles with neighbour lists ngb and
 * smoothing lengths h (as produced by sidm_find_ngb), timesteps dt[n_active],
 * Philox seed and step counter.  Velocities (and state) of every kicked
 * particle are written to p's arrays, which must be the arrays given to
 * sidm_build_tree.  cand_info (optional, [n_active*n_ngb]) receives the
 * SIDM_CAND_* bits and pass index of every candidate. */
sidm_status sidm_scatter_step(sidm_ctx *ctx, sidm_particles *p, const int32_t *active,
                              int64_t n_active, const int32_t *ngb, const double *h,
                              const double *dt, uint64_t seed, uint32_t step,
                              uint32_t *cand_info);

/* dt_sidm[a] = c_sidm * 2 / (m_i W(0, h_a) max_{j in N(i)} w_ij sigma(w_ij)/m) with
 * the current (post-kick) velocities; +inf when the maximum is 0. */
sidm_status sidm_pair_timestep(sidm_ctx *ctx, const int32_t *active, int64_t n_active,
                               const int32_t *ngb, const double *h, double *dt_sidm);

/* ---- Kernel-overlap estimator (Eq. kernelOverlap; the paper's appendix on
 * the overlap kernel) -------------------------------------------------------
 * g_ij is the overlap integral of the two particles' cubic splines,
 * int W(|x - x_i|, h_i) W(|x - x_j|, h_j) d^3x, non-zero for r_ij < h_i + h_j.
 * These calls need a context created with estimator SIDM_EST_OVERLAP
 * (SIDM_E_STATE otherwise) and a sidm_build_tree of the current positions.
 * h_all[n] (device, caller order) holds every particle's smoothing length,
 * active or not (> 0 and finite; for example sidm_find_ngb's h over all
 * particles, or the last value of those not active now). */

/* Partners of the active particles.  If h_active is not NULL, it holds the
 * new smoothing lengths of the active particles (h_active[a] for active[a],
 * for example sidm_find_ngb's h) and is first written into h_all, which is
 * then read as every particle's h (so h_all is in/out).  For active[a] = i,
 * the partners are every j != i with
 * r_ij < h_i + h_j, tested as r^2 < (h_i + h_j)^2 in FP64 with r^2 as in
 * sidm_find_ngb.  The tree's nodes first get the largest h below them (the
 * search region is h_i + that h_max).  Row a of ngb (max_ngb >= 1 entries,
 * caller indices) receives min(count[a], max_ngb) partners in an order fixed
 * by the tree (not sorted), count[a] their full number.  A row longer than
 * max_ngb keeps its first max_ngb and latches SIDM_E_OVERFLOW (sidm_sync);
 * an h that is not > 0 and finite latches SIDM_E_INVAL. */
sidm_status sidm_find_overlap(sidm_ctx *ctx, double *h_all, const int32_t *active,
                              const double *h_active, int64_t n_active, int32_t max_ngb,
                              int32_t *ngb, int32_t *count);

/* Scattering step with the overlap estimator: sidm_scatter_step with the
 * partners of row a being the first min(count[a], max_ngb) entries of
 * ngb[a*max_ngb ...] (rows as sidm_find_overlap writes them; their order does
 * not matter) and, in place of W(r_ij, h_i),
 *     g_ij = ghat(alpha, rho) / H^3,  H = h_i + h_j,
 *     alpha = min(h_i, h_j) / H,  rho = r_ij / H,
 * with ghat(alpha, rho) = H^3 g at h_i = alpha H, h_j = (1 - alpha) H (the
 * pair symmetry g_ij = g_ji leaves alpha in [0, 1/2]; alpha = 0 is a point
 * partner, ghat = W(rho, 1)) computed at the table nodes when the context is
 * created and read bilinearly: with fa = alpha 2 NA, fr = rho NR,
 * ia = min(floor(fa), NA-1), ir = min(floor(fr), NR-1), ta = fa - ia,
 * tr = fr - ir:  g0 = T[ia][ir] + tr (T[ia][ir+1] - T[ia][ir]),
 * g1 likewise from row ia+1,  ghat = g0 + ta (g1 - g0);  0 for rho >= 1.
 * h_all as given to sidm_find_overlap (the Morton-order copy of it that the
 * call made is read while the tree and the h_all address are unchanged,
 * else gathered again); cand_info (optional) has n_active*max_ngb entries,
 * slot a*max_ngb + s. */
sidm_status sidm_scatter_overlap(sidm_ctx *ctx, sidm_particles *p, const double *h_all,
                                 const int32_t *active, int64_t n_active, int32_t max_ngb,
                                 const int32_t *ngb, const int32_t *count, const double *dt,
                                 uint64_t seed, uint32_t step, uint32_t *cand_info);

/* Per-pair timestep with the overlap estimator: Eq. sidm_timestep with the
 * kernel's centre value W(0, h_i) replaced by each pair's g_ij at zero
 * separation (the largest value g_ij takes):
 *     dt_sidm[a] = c_sidm * 2 / (m_i max_j [g_ij(0) (w_ij sigma(w_ij)/m)])
 * over the partners of row a, with the current velocities; +inf if 0.
 * h_all as for sidm_scatter_overlap. */
sidm_status sidm_pair_timestep_overlap(sidm_ctx *ctx, const double *h_all, const int32_t *active,
                                       int64_t n_active, int32_t max_ngb, const int32_t *ngb,
                                       const int32_t *count, double *dt_sidm);

/* Copy the context's ghat table, (NA+1) x (NR+1) doubles alpha-major, to
 * HOST memory host_out (waits for the context's stream). */
sidm_status sidm_overlap_table(sidm_ctx *ctx, double *host_out);

/* Served form: the step between two scattering steps of an isolated halo
 * that has no gravity solver of its own.  The step length d is the largest
 * dt_cap / 2^b (b >= 0) not above min(dt_sidm[0..n_active)) -- the per-pair
 * bounds sidm_pair_timestep just wrote (sec. 4.4) -- or dt_cap if
 * n_active == 0.  d is written to dt_next[0..n_active) (the dt of the next
 * sidm_scatter_step; may be NULL) and to *dt_step (device scalar; may be
 * NULL).  Then all n particles take one kick-drift-kick step of length d in
 * the Hernquist potential Phi(r) = -gm / (r + a) (positions and velocities
 * updated in place; caller-owned device arrays of n doubles each).  Needs
 * dt_cap > 0, gm >= 0, a > 0, n <= cap_n; asynchronous on the context's
 * stream, no allocation. */
sidm_status sidm_advance_hernquist(sidm_ctx *ctx, double *x, double *y, double *z, double *vx,
                                   double *vy, double *vz, int64_t n, const double *dt_sidm,
                                   int64_t n_active, double dt_cap, double gm, double a,
                                   double *dt_next, double *dt_step);

/* Allocation-free form of sidm_advance_hernquist, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  It needs no context: the same step
 * (same arguments and results, bit for bit) on the current HIP device and on
 * `hip_stream` (hipStream_t, may be NULL).  The reduction's partial minima
 * live in a fixed device array of the library (4097 64-bit words, 32 KiB,
 * one copy per GPU held until the process ends), so n_active is limited to
 * 8,388,608 (SIDM_E_CAPACITY above it, before anything is enqueued; other
 * argument errors SIDM_E_INVAL as for sidm_advance_hernquist, n <= 2^31 - 1).
 * The call allocates nothing and clears nothing with hipMemset: every word
 * of the array it reads it first writes.  Calls that overlap on one GPU
 * (different streams, or host threads) share that array and race: order
 * them on one stream.  SIDM_E_DEVICE if a launch fails. */
sidm_status sidm_advance_hernquist_noalloc(void *hip_stream, double *x, double *y, double *z,
                                           double *vx, double *vy, double *vz, int64_t n,
                                           const double *dt_sidm, int64_t n_active,
                                           double dt_cap, double gm, double a,
                                           double *dt_next, double *dt_step);

/* Free drift between scattering steps of a box without gravity (the
 * thermalisation box of sec. 5.2): x += v dt for all n particles, wrapped
 * into [0, box) when the configuration is periodic.  Caller-owned device
 * arrays of n doubles; needs a finite dt >= 0 and n <= cap_n; asynchronous on
 * the context's stream, no allocation. */
sidm_status sidm_drift(sidm_ctx *ctx, double *x, double *y, double *z, const double *vx,
                       const double *vy, const double *vz, int64_t n, double dt);

/* Wait for the context's stream, copy the statistics of the last
 * sidm_scatter_step into *out (may be NULL) and return the latched device
 * error (SIDM_OK if none).  Clears the latched error. */
sidm_status sidm_sync(sidm_ctx *ctx, sidm_stats *out);

/* ---- Measurement (not part of the method) --------------------------------
 * sidm_timing_enable(ctx, phases) brackets the launches of the phases in the
 * mask (SIDM_TIMING_*; 0 turns timing off) with HIP events on the context's
 * stream, up to 256 launches of each between two reads; it restarts the
 * window.  Each bracketed phase leaves the GPU idle for a few microseconds at
 * its two ends, so time only the phases needed.  sidm_timing_read waits for
 * the stream, reports the mean device time in milliseconds of the launches
 * since the previous read (or enable) of each timed phase (0 for the others)
 * and starts a new window.  Disabled by default; a mask with other bits is
 * SIDM_E_INVAL. */
#define SIDM_TIMING_TREE 1
#define SIDM_TIMING_MAP 2
#define SIDM_TIMING_KNN 4
#define SIDM_TIMING_EVAL 8
#define SIDM_TIMING_RESOLVE 16
#define SIDM_TIMING_TIMESTEP 32
#define SIDM_TIMING_OVERLAP 64
#define SIDM_TIMING_ALL 127
typedef struct {
    int32_t samples;      /* neighbour-search launches averaged                    */
    int32_t pad;
    double tree_ms;       /* sidm_build_tree: every kernel of the build            */
    double map_ms;        /* active-list mapping of the most recent call           */
    double knn_ms;        /* the neighbour-search kernel                           */
    double eval_ms;       /* the candidate-evaluation kernel                       */
    double resolve_ms;    /* all resolution passes (grid passes and finisher)      */
    double timestep_ms;   /* the per-pair timestep kernel                          */
    double overlap_ms;    /* sidm_find_overlap: h update, node h_max and the walk  */
} sidm_timing;

sidm_status sidm_timing_enable(sidm_ctx *ctx, int phases);
sidm_status sidm_timing_read(sidm_ctx *ctx, sidm_timing *out);

#ifdef __cplusplus
}
#endif
#endif /* SIDM_H */
