/*
 * sidm_oracle.c -- plain, slow, FP64 CPU reference of one SIDM scattering step
 * (Zier et al., "A Novel Implementation of Self-Interacting Dark Matter in
 * AREPO", arXiv 2607.05504).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is
 * checked against.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library neither
 * includes, links nor calls anything here, and this file includes nothing of
 * the GPU library.  Build:  gcc -O2 -ffp-contract=off -fno-fast-math -shared
 * -fPIC (no FMA contraction, so every expression rounds exactly as written).
 *
 * What is computed, in the paper's order (section numbers are the paper's):
 *   separation      minimum-image offset in a periodic box (sec. 5.2 uses a
 *                   periodic box; the convention is this oracle's reading)
 *   neighbours      the N_ngb nearest DM particles of each active target,
 *                   inactive ones included (sec. 4.1, Fig. 3 caption);
 *                   smoothing length h_i = distance of the (N_ngb+1)-th
 *                   (reading of the "32 +- 5" bisection of sec. 4.2/4.5)
 *   kernel          cubic spline W_CS(q, h) (sec. 4.2)
 *   cross-section   sigma/m constant, or s0 / (1 + (w/w0)^2)^2 (sec. 5.2),
 *                   or a table interpolated linearly in log velocity (sec. 4.2)
 *   units           separations, smoothing lengths and relative speeds are
 *                   converted to physical units by two factors before they
 *                   enter W, g_ij, sigma, P, the two-state balance and dt
 *                   (sec. 4.2: comoving storage, physical pair rate)
 *   rate, P         Gamma(i|j) = m_j (sigma/m) |v_i - v_j| g_ij with the
 *                   one-sided g_ij = W(x_j - x_i, h_i)   (Eqs. rate, oneSided)
 *                   P(i|j) = Gamma(i|j) dt_i / 2        (Eq. probabilityScatter)
 *   random numbers  Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11),
 *                   keyed on the seed, counter = (lower ID, higher ID, step,
 *                   purpose) -- the paper only says a random number is drawn
 *   acceptance      every directed candidate (i|j) takes one turn, in
 *                   increasing (priority, id_i, id_j) with a Philox priority;
 *                   at its turn P is computed with the velocities as they are
 *                   then, so a pair evaluated after a kick of one of its
 *                   particles sees the kicked velocity (sec. 4.5, immediate
 *                   update), and it scatters iff u < P
 *   kick            centre-of-momentum kick with a direction uniform on the
 *                   sphere and outgoing relative speed eps * w (sec. 4.1);
 *                   eps = 1 elastic, constant eps, or a two-state model whose
 *                   eps follows from the energy gap (sec. 4.1 relates eps to
 *                   the energy released or absorbed); or the fixed-target
 *                   beam test of sec. 5.1 (no recoil of the target)
 *   timestep        dt_i = C_SIDM * 2 / (m_DM W(0, h_i) (v sigma/m)_max)
 *                   (Eq. sidm_timestep)
 *   overlap         the kernel-overlap estimator (Eq. kernelOverlap and the
 *                   appendix on it): partners are all j with
 *                   r_ij < h_i + h_j, and g_ij is the overlap integral of the
 *                   two splines, read from a table of the dimensionless
 *                   overlap ghat(h_i/(h_i+h_j), r_ij/(h_i+h_j))
 *
 * Built with -fopenmp as well (a second library, the CPU throughput
 * baseline): the loops over targets of the neighbour ranking, of the
 * step-start evaluation and of the timestep then run on all cores; the turns
 * stay one after another, so the results are the same bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OREF_PI 3.14159265358979323846
#define OREF_OK 0
#define OREF_E_INVAL -1
#define OREF_E_NOMEM -2

/* scatter models / cross-sections (integer values shared with the Python side) */
#define OREF_XSEC_CONST 0
#define OREF_XSEC_YUKAWA 1
#define OREF_XSEC_TABLE 2
#define OREF_TABLE_MAX 256
#define OREF_MODEL_ELASTIC 0
#define OREF_MODEL_EPS 1
#define OREF_MODEL_TWO_STATE 2
#define OREF_MODEL_BEAM 3        /* fixed-target beam test (sec. 5.1): state 1 = beam,
                                    0 = target; only beam-target pairs scatter and
                                    the target does not recoil */

/* per-candidate info word */
#define OREF_CAND_ACCEPT0 1u   /* u < P with the step-start velocities (diagnostic) */
#define OREF_CAND_SCATTER 2u   /* produced a kick at its turn                       */
#define OREF_CAND_FLAGGED 4u   /* |P - u| < band at its turn                        */
/* bits 8..31: a kick's depth in the chain of kicks (0: no kick) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 S-box with the   */
/* multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9,     */
/* 0xBB67AE85.                                                                 */
/* ------------------------------------------------------------------------ */
void oref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* purposes of a draw for one unordered pair in one step */
#define PURPOSE_DECIDE 0u
#define PURPOSE_DIR_LO_HI 1u
#define PURPOSE_PRIORITY 2u
#define PURPOSE_DIR_HI_LO 3u

static void pair_draw(uint64_t seed, uint32_t step, uint32_t id_a, uint32_t id_b,
                      uint32_t purpose, uint32_t out[4])
{
    uint32_t lo = id_a < id_b ? id_a : id_b;
    uint32_t hi = id_a < id_b ? id_b : id_a;
    uint32_t ctr[4] = {lo, hi, step, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oref_philox4x32_10(ctr, key, out);
}

/* The 64-bit word serving the direction "target -> partner": words (x0,x1)
 * serve the lower-ID target, (x2,x3) the higher-ID target. */
static uint64_t direction_word(const uint32_t x[4], int target_is_lower)
{
    return target_is_lower ? ((uint64_t)x[1] << 32 | x[0]) : ((uint64_t)x[3] << 32 | x[2]);
}

static double unit_from_word(uint64_t w)
{
    return (double)(w >> 11) * 0x1.0p-53;   /* in [0, 1) */
}

double oref_uniform_decision(uint64_t seed, uint32_t step, uint32_t id_i, uint32_t id_j)
{
    uint32_t x[4];
    pair_draw(seed, step, id_i, id_j, PURPOSE_DECIDE, x);
    return unit_from_word(direction_word(x, id_i < id_j));
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* one axis of the separation x_j - x_i, minimum image when periodic */
static double axis_sep(double xi, double xj, int periodic, double box)
{
    double d = xj - xi;
    if (periodic) {
        if (d >= 0.5 * box) d = d - box;
        else if (d < -0.5 * box) d = d + box;
    }
    return d;
}

double oref_r2(double xi, double yi, double zi, double xj, double yj, double zj,
               int periodic, double box)
{
    double dx = axis_sep(xi, xj, periodic, box);
    double dy = axis_sep(yi, yj, periodic, box);
    double dz = axis_sep(zi, zj, periodic, box);
    return (dx * dx + dy * dy) + dz * dz;
}

/* cubic spline kernel with compact support h (sec. 4.2) */
double oref_kernel(double r, double h)
{
    double h3 = (h * h) * h;
    double norm = 8.0 / (OREF_PI * h3);
    double q = r / h;
    if (q <= 0.5) {
        double q2 = q * q;
        double q3 = q2 * q;
        return norm * ((1.0 - 6.0 * q2) + 6.0 * q3);
    }
    if (q <= 1.0) {
        double t = 1.0 - q;
        return norm * (2.0 * ((t * t) * t));
    }
    return 0.0;
}

/* Stored -> physical units (sec. 4.2: in cosmological runs coordinates and
 * velocities are comoving, and the pair rate is evaluated in physical units,
 * separations and smoothing lengths times one factor, relative speeds times
 * another; both 1 for physical storage), set by oref_set_units. */
static double oref_len = 1.0, oref_vel = 1.0;

int oref_set_units(double len_to_phys, double vel_to_phys)
{
    if (!(len_to_phys > 0.0) || !(len_to_phys < 1e300) || !(vel_to_phys > 0.0) ||
        !(vel_to_phys < 1e300))
        return OREF_E_INVAL;
    oref_len = len_to_phys;
    oref_vel = vel_to_phys;
    return OREF_OK;
}

/* tabulated cross-section: node speeds (increasing) and values, set by
 * oref_set_table before a step that uses it */
static double oref_tw[OREF_TABLE_MAX], oref_ts[OREF_TABLE_MAX];
static int oref_tn = 0;

int oref_set_table(const double *w, const double *s, int n)
{
    if (n < 2 || n > OREF_TABLE_MAX) return OREF_E_INVAL;
    for (int q = 0; q < n; ++q) {
        if (!(w[q] > 0.0) || (q > 0 && !(w[q] > w[q - 1])) || !(s[q] >= 0.0)) return OREF_E_INVAL;
        oref_tw[q] = w[q];
        oref_ts[q] = s[q];
    }
    oref_tn = n;
    return OREF_OK;
}

/* sigma/m of the table at speed w (sec. 4.2: linear interpolation in log
 * velocity): the end value outside the nodes, else the straight line in ln w
 * through the two nodes that bracket w (tw[k] <= w < tw[k+1]), found here by
 * a linear scan */
static double oref_sigma_table(double w)
{
    const int n = oref_tn;
    if (!(w > oref_tw[0])) return oref_ts[0];
    if (!(w < oref_tw[n - 1])) return oref_ts[n - 1];
    int k = 0;
    while (!(oref_tw[k + 1] > w)) ++k;
    const double lo = log(oref_tw[k]), hi = log(oref_tw[k + 1]);
    const double f = (log(w) - lo) / (hi - lo);
    return oref_ts[k] + f * (oref_ts[k + 1] - oref_ts[k]);
}

double oref_sigma(double w, int xsec, double s0, double w0)
{
    if (xsec == OREF_XSEC_TABLE) return oref_sigma_table(w);
    if (xsec == OREF_XSEC_YUKAWA) {
        double x = w / w0;
        double d = 1.0 + x * x;
        return s0 / (d * d);
    }
    return s0;
}

static double rel_speed(double ax, double ay, double az, double bx, double by, double bz)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

/* P(i|j) = 1/2 m_j (sigma(w)/m) w W dt_i, multiplied left to right */
static double pair_probability(double m_j, double sig, double w, double W, double dt)
{
    return (((0.5 * m_j) * sig) * w * W) * dt;
}

/* ------------------------------------------------------------------------ */
/* Neighbours: for each target i, all j != i ordered by (r2_ij, id_j); the    */
/* first k are N(i) and h_i = sqrt(r2 of entry k+1).                          */
/* ------------------------------------------------------------------------ */
typedef struct { double r2; uint32_t id; int32_t j; } cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->r2 < b->r2) return -1;
    if (a->r2 > b->r2) return 1;
    if (a->id < b->id) return -1;
    if (a->id > b->id) return 1;
    return 0;
}

/*
 * n particles; targets[n_t] indices; k = N_ngb.
 * cand_ptr/cand_idx: optional CSR superset of candidate partners per target
 * (NULL: every particle).  A superset must contain every j with r2_ij <= the
 * true (k+1)-th smallest value; the ranking below does not depend on it.
 * Out: ngb[n_t*k] (row-major, sorted by (r2, id)), h[n_t].
 */
int oref_find_ngb(int64_t n, const double *x, const double *y, const double *z,
                  const uint32_t *id, int periodic, double box,
                  int64_t n_t, const int32_t *targets, int k,
                  const int64_t *cand_ptr, const int32_t *cand_idx,
                  int32_t *ngb, double *h)
{
    if (k < 1 || n < k + 2) return OREF_E_INVAL;
    int64_t cap = n;             /* longest candidate row */
    if (cand_ptr) {
        cap = 1;
        for (int64_t t = 0; t < n_t; ++t)
            if (cand_ptr[t + 1] - cand_ptr[t] > cap) cap = cand_ptr[t + 1] - cand_ptr[t];
    }
    int rc = OREF_OK;
#pragma omp parallel
    {
        cand_t *buf = (cand_t *)malloc((size_t)cap * sizeof(cand_t));
        if (!buf) {
#pragma omp atomic write
            rc = OREF_E_NOMEM;
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t t = 0; t < n_t; ++t) {
            if (!buf) continue;
            int32_t i = targets[t];
            int64_t m = 0;
            int64_t lo = cand_ptr ? cand_ptr[t] : 0;
            int64_t hi = cand_ptr ? cand_ptr[t + 1] : n;
            for (int64_t c = lo; c < hi; ++c) {
                int32_t j = cand_ptr ? cand_idx[c] : (int32_t)c;
                if (j == i) continue;
                buf[m].r2 = oref_r2(x[i], y[i], z[i], x[j], y[j], z[j], periodic, box);
                buf[m].id = id[j];
                buf[m].j = j;
                ++m;
            }
            if (m < k + 1) {
#pragma omp atomic write
                rc = OREF_E_INVAL;
                continue;
            }
            qsort(buf, (size_t)m, sizeof(cand_t), cand_cmp);
            for (int s = 0; s < k; ++s) ngb[t * k + s] = buf[s].j;
            h[t] = sqrt(buf[k].r2);
        }
        free(buf);
    }
    return rc;
}

/* The order in which the scatter step visits the turns (the result is the
 * same): 0 visits every candidate in order; 1 visits, in the same order, only
 * the candidates whose turn can differ from their step-start evaluation --
 * those accepted at the step start and those touching a particle kicked
 * earlier in the order.  Every other candidate meets both of its particles
 * unkicked at its turn, so its P and decision are the step-start ones.  1
 * exists for steps of many millions of candidates; tests pin it to 0. */
static int oref_turn_mode = 0;
int oref_set_turn_mode(int mode)
{
    if (mode == 0 || mode == 1) oref_turn_mode = mode;
    return oref_turn_mode;
}

/* threads of the OpenMP build (want > 0 sets them); 1 for the plain build */
int oref_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) omp_set_num_threads(want);
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Kick (sec. 4.1): v' = v_com +- eps m_other |v_i - v_j| / (m_i + m_j) e     */
/* ------------------------------------------------------------------------ */
static void direction_from_draw(const uint32_t x[4], double e[3])
{
    uint64_t wa = (uint64_t)x[1] << 32 | x[0];
    uint64_t wb = (uint64_t)x[3] << 32 | x[2];
    double u1 = unit_from_word(wa), u2 = unit_from_word(wb);
    double cth = 2.0 * u1 - 1.0;
    double phi = 2.0 * OREF_PI * u2;
    double s2 = 1.0 - cth * cth;
    double sth = sqrt(s2 > 0.0 ? s2 : 0.0);
    e[0] = sth * cos(phi);
    e[1] = sth * sin(phi);
    e[2] = cth;
}

typedef struct {
    int xsec; double s0, w0;
    int model; double eps, delta;
    uint64_t seed; uint32_t step;
} phys_t;

/* Returns the outgoing/incoming relative-speed ratio and the state changes of
 * the scatter of particles a (target) and b, for the chosen model. */
static double scatter_eps(const phys_t *ph, double m_a, double m_b, double w,
                          uint8_t s_a, uint8_t s_b, uint32_t id_a, uint32_t id_b,
                          uint32_t channel_bit, uint8_t *ns_a, uint8_t *ns_b)
{
    *ns_a = s_a; *ns_b = s_b;
    if (ph->model == OREF_MODEL_EPS) return ph->eps;
    if (ph->model != OREF_MODEL_TWO_STATE) return 1.0;
    /* two-state: energy gap delta per unit mass of the particle changing state.
     * Centre-of-momentum kinetic energy (1/2) mu w^2 changes by -dE:
     *   eps^2 = 1 - 2 dE / (mu w^2),  dE = +m_p delta (excite), -m_p delta (de-excite). */
    double M = m_a + m_b;
    double mu = (m_a * m_b) / M;
    int a_is_lower = id_a < id_b;
    if (s_a == 0 && s_b == 0) {
        /* excite the lower-ID particle when the channel bit is 0, else the higher */
        int excite_a = (channel_bit == 0) ? a_is_lower : !a_is_lower;
        double m_p = excite_a ? m_a : m_b;
        double e2 = 1.0 - (2.0 * m_p * ph->delta) / ((mu * w) * w);
        if (!(e2 > 0.0)) return 1.0;               /* below threshold: elastic */
        if (excite_a) *ns_a = 1; else *ns_b = 1;
        return sqrt(e2);
    }
    int deexcite_a;
    if (s_a && s_b) deexcite_a = (channel_bit == 0) ? a_is_lower : !a_is_lower;
    else deexcite_a = s_a != 0;
    double m_p = deexcite_a ? m_a : m_b;
    double e2 = 1.0 + (2.0 * m_p * ph->delta) / ((mu * w) * w);
    if (deexcite_a) *ns_a = 0; else *ns_b = 0;
    return sqrt(e2);
}

static void do_kick(const phys_t *ph, int32_t i, int32_t j, const double *mass, double m_scalar,
                    double *vx, double *vy, double *vz, uint8_t *state, const uint32_t *id)
{
    if (ph->model == OREF_MODEL_BEAM) {
        /* no recoil: the target (state 0) is the infinitely heavy limit of the
         * kick below -- its velocity stays, the beam particle's velocity
         * relative to it turns to the drawn direction with unchanged speed
         * (+e if the beam particle is the candidate's target i, -e if it is j) */
        uint32_t xb[4];
        pair_draw(ph->seed, ph->step, id[i], id[j],
                  id[i] < id[j] ? PURPOSE_DIR_LO_HI : PURPOSE_DIR_HI_LO, xb);
        double eb[3];
        direction_from_draw(xb, eb);
        double w = rel_speed(vx[i], vy[i], vz[i], vx[j], vy[j], vz[j]);
        if (state[i] == 1) {
            vx[i] = vx[j] + w * eb[0]; vy[i] = vy[j] + w * eb[1]; vz[i] = vz[j] + w * eb[2];
        } else {
            vx[j] = vx[i] - w * eb[0]; vy[j] = vy[i] - w * eb[1]; vz[j] = vz[i] - w * eb[2];
        }
        return;
    }
    double mi = mass ? mass[i] : m_scalar;
    double mj = mass ? mass[j] : m_scalar;
    uint32_t x[4];
    /* direction draw: purpose 1 serves the lower-ID target, 3 the higher-ID one */
    pair_draw(ph->seed, ph->step, id[i], id[j],
              id[i] < id[j] ? PURPOSE_DIR_LO_HI : PURPOSE_DIR_HI_LO, x);
    double e[3];
    direction_from_draw(x, e);
    double w = rel_speed(vx[i], vy[i], vz[i], vx[j], vy[j], vz[j]);
    uint8_t si = state ? state[i] : 0, sj = state ? state[j] : 0, nsi, nsj;
    /* the energy balance in physical speed; the kick itself in stored units */
    double eps = scatter_eps(ph, mi, mj, oref_vel * w, si, sj, id[i], id[j], x[0] & 1u, &nsi,
                             &nsj);
    double M = mi + mj;
    double vcx = (mi * vx[i] + mj * vx[j]) / M;
    double vcy = (mi * vy[i] + mj * vy[j]) / M;
    double vcz = (mi * vz[i] + mj * vz[j]) / M;
    double c = (eps * w) / M;
    double ci = mj * c, cj = mi * c;
    vx[i] = vcx + ci * e[0]; vy[i] = vcy + ci * e[1]; vz[i] = vcz + ci * e[2];
    vx[j] = vcx - cj * e[0]; vy[j] = vcy - cj * e[1]; vz[j] = vcz - cj * e[2];
    if (state) { state[i] = nsi; state[j] = nsj; }
}

/* ------------------------------------------------------------------------ */
/* Scatter step (sec. 4.1, 4.5)                                              */
/* ------------------------------------------------------------------------ */
/* one directed candidate (i|j): its place in the serial order and its slot */
typedef struct {
    uint64_t prio;      /* priority word of the pair draw */
    uint32_t id_i, id_j;
    int64_t c;          /* candidate slot a*stride + s */
    int64_t a;          /* its row */
} cand_ord_t;

static int cand_ord_cmp(const void *pa, const void *pb)
{
    const cand_ord_t *a = (const cand_ord_t *)pa, *b = (const cand_ord_t *)pb;
    if (a->prio != b->prio) return a->prio < b->prio ? -1 : 1;
    if (a->id_i != b->id_i) return a->id_i < b->id_i ? -1 : 1;
    if (a->id_j != b->id_j) return a->id_j < b->id_j ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t n_cand, n_accept0, n_events, n_flagged, n_p_ge_1;
    int32_t n_passes; double max_p;
} oref_stats;

double oref_overlap_g(double hi, double hj, double r);

/* W (one-sided spline or tabulated overlap) and P of candidate slot ci of row
 * a with the velocities as they are now; all lengths and the relative speed
 * in physical units */
static double candidate_probability(const double *x, const double *y, const double *z,
                                    const double *vx, const double *vy, const double *vz,
                                    const double *mass, double m_scalar, const uint8_t *state,
                                    int periodic, double box, int32_t i, int32_t j,
                                    const double *h, const double *h_all, int64_t a,
                                    const double *dt, int xsec, double s0, double w0, int model)
{
    double r = oref_len * sqrt(oref_r2(x[i], y[i], z[i], x[j], y[j], z[j], periodic, box));
    double W = h_all ? oref_overlap_g(oref_len * h_all[i], oref_len * h_all[j], r)
                     : oref_kernel(r, oref_len * h[a]);
    double w = oref_vel * rel_speed(vx[i], vy[i], vz[i], vx[j], vy[j], vz[j]);
    double sig = oref_sigma(w, xsec, s0, w0);
    double mj = mass ? mass[j] : m_scalar;
    double P = pair_probability(mj, sig, w, W, dt[a]);
    if (model == OREF_MODEL_BEAM && state[i] == state[j]) P = 0.0;
    return P;
}

/* Min-heap of turns in cand_ord_cmp order (the event-driven visit). */
typedef struct { cand_ord_t *e; int64_t n, cap; } turn_heap;

static int heap_push(turn_heap *h, cand_ord_t v)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        cand_ord_t *ne = (cand_ord_t *)realloc(h->e, (size_t)nc * sizeof(cand_ord_t));
        if (!ne) return -1;
        h->e = ne; h->cap = nc;
    }
    int64_t q = h->n++;
    while (q > 0) {
        int64_t p = (q - 1) / 2;
        if (cand_ord_cmp(&h->e[p], &v) <= 0) break;
        h->e[q] = h->e[p];
        q = p;
    }
    h->e[q] = v;
    return 0;
}

static cand_ord_t heap_pop(turn_heap *h)
{
    cand_ord_t top = h->e[0], last = h->e[--h->n];
    int64_t q = 0;
    for (;;) {
        int64_t c = 2 * q + 1;
        if (c >= h->n) break;
        if (c + 1 < h->n && cand_ord_cmp(&h->e[c + 1], &h->e[c]) < 0) ++c;
        if (cand_ord_cmp(&last, &h->e[c]) <= 0) break;
        h->e[q] = h->e[c];
        q = c;
    }
    if (h->n > 0) h->e[q] = last;
    return top;
}

/* row of dense candidate index d (row_off[a] <= d < row_off[a + 1]) */
static int64_t row_of(const int64_t *row_off, int64_t n_active, int64_t d)
{
    int64_t lo = 0, hi = n_active - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (row_off[mid] <= d) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/*
 * Shared by both estimators.  Row a of ngb (stride entries) holds the
 * partners of active[a]; count[a] of them are used (all stride when count is
 * NULL).  The geometric factor is W(r_ij, h[a]) (one-sided), or the
 * tabulated overlap of h_all[i] and h_all[j] when h_all is given.
 *
 * Sec. 4.5: pairs are processed one after another, and a pair evaluated after
 * a kick of one of its particles sees the kicked velocity (immediate update).
 * The paper's order is that of its loop over particles and tasks; here every
 * directed candidate (i|j) takes its turn in increasing (priority, id_i,
 * id_j), the priority being a Philox word of the pair, so the order does not
 * depend on storage.  At its turn a candidate's P is computed with the
 * current velocities and it scatters iff u < P, u its own decision draw;
 * every candidate has exactly one turn.
 *
 * v and state are updated in place.  cand_info[n_active*stride] (optional):
 * ACCEPT0 if u < P with the step-start velocities (a diagnostic), FLAGGED if
 * |P - u| < band at its turn, SCATTER if it kicked, and for a kick its depth
 * in bits 8..31: 1 + the larger depth of the last earlier kicks of its two
 * particles (0 for a particle not yet kicked), i.e. the round in which a
 * parallel matching of the kicks in this order would apply it.  Stats:
 * n_accept0, n_p_ge_1 and max_p of the step-start evaluation; n_events kicks;
 * n_flagged flagged turns; n_passes the largest depth.
 */
/* The scatter step visiting only the turns that can differ from their
 * step-start evaluation (oref_turn_mode 1; see oref_set_turn_mode).  Same
 * arguments as scatter_core, plus its row offsets. */
static int scatter_events(int64_t n, const double *x, const double *y, const double *z,
                          double *vx, double *vy, double *vz, const double *mass, double m_scalar,
                          const uint32_t *id, uint8_t *state, int periodic, double box,
                          int64_t n_active, const int32_t *active, int stride,
                          const int32_t *ngb, const double *h, const double *h_all, const double *dt,
                          const phys_t *ph, double band, const int64_t *row_off, int64_t n_cand,
                          uint32_t *cand_info, oref_stats *st)
{
    enum { F_ACC0 = 1, F_FLAG0 = 2, F_QUEUED = 4, F_FLAGT = 8 };
    const int xsec = ph->xsec, model = ph->model;
    const double s0 = ph->s0, w0 = ph->w0;
    const uint64_t seed = ph->seed;
    const uint32_t step = ph->step;
    uint8_t *fl = (uint8_t *)calloc((size_t)(n_cand > 0 ? n_cand : 1), 1);
    int32_t *a_of = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *rstart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *rlist = (int64_t *)malloc((size_t)(n_cand > 0 ? n_cand : 1) * sizeof(int64_t));
    int32_t *depth = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    turn_heap hp = {NULL, 0, 0};
    int rc = OREF_OK;
    if (!fl || !a_of || !rstart || !rlist || !depth) { rc = OREF_E_NOMEM; goto done; }

    /* step-start evaluation of every candidate */
    double max_p = 0.0;
    int64_t n_ge1 = 0, n_acc0 = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : max_p) reduction(+ : n_ge1, n_acc0)
    for (int64_t a = 0; a < n_active; ++a) {
        int32_t i = active[a];
        for (int64_t d = row_off[a]; d < row_off[a + 1]; ++d) {
            int64_t ci = a * (int64_t)stride + (d - row_off[a]);
            int32_t j = ngb[ci];
            double P = candidate_probability(x, y, z, vx, vy, vz, mass, m_scalar, state, periodic,
                                             box, i, j, h, h_all, a, dt, xsec, s0, w0, model);
            double u = oref_uniform_decision(seed, step, id[i], id[j]);
            if (P > max_p) max_p = P;
            if (P >= 1.0) n_ge1++;
            uint8_t f = 0;
            if (u < P) { f |= F_ACC0; n_acc0++; }
            if (fabs(P - u) < band) f |= F_FLAG0;
            fl[d] = f;
        }
    }
    st->max_p = max_p;
    st->n_p_ge_1 = n_ge1;
    st->n_accept0 = n_acc0;

    /* the candidates touching each particle: its own row, and the rows that
     * list it (a reverse index of the partners) */
    for (int64_t p = 0; p < n; ++p) a_of[p] = -1;
    for (int64_t a = 0; a < n_active; ++a) a_of[active[a]] = (int32_t)a;
    for (int64_t a = 0; a < n_active; ++a)
        for (int64_t d = row_off[a]; d < row_off[a + 1]; ++d)
            rstart[ngb[a * (int64_t)stride + (d - row_off[a])] + 1]++;
    for (int64_t p = 0; p < n; ++p) rstart[p + 1] += rstart[p];
    {
        int64_t *cur = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!cur) { rc = OREF_E_NOMEM; goto done; }
        memcpy(cur, rstart, (size_t)n * sizeof(int64_t));
        for (int64_t a = 0; a < n_active; ++a)
            for (int64_t d = row_off[a]; d < row_off[a + 1]; ++d)
                rlist[cur[ngb[a * (int64_t)stride + (d - row_off[a])]]++] = d;
        free(cur);
    }

    /* a turn's key, as the plain order sorts it */
#define TURN_OF(D, A, OUT)                                                              \
    do {                                                                               \
        int64_t ci_ = (A) * (int64_t)stride + ((D) - row_off[A]);                      \
        int32_t i_ = active[A], j_ = ngb[ci_];                                         \
        uint32_t xr_[4];                                                               \
        pair_draw(seed, step, id[i_], id[j_], PURPOSE_PRIORITY, xr_);                   \
        cand_ord_t e_ = {direction_word(xr_, id[i_] < id[j_]), id[i_], id[j_], ci_, (A)}; \
        (OUT) = e_;                                                                    \
    } while (0)

    for (int64_t a = 0; a < n_active; ++a)
        for (int64_t d = row_off[a]; d < row_off[a + 1]; ++d)
            if (fl[d] & F_ACC0) {
                cand_ord_t e;
                TURN_OF(d, a, e);
                fl[d] |= F_QUEUED;
                if (heap_push(&hp, e)) { rc = OREF_E_NOMEM; goto done; }
            }
    while (hp.n > 0) {
        cand_ord_t c = heap_pop(&hp);
        int32_t i = active[c.a], j = ngb[c.c];
        int64_t dc = row_off[c.a] + (c.c - c.a * (int64_t)stride);
        double P = candidate_probability(x, y, z, vx, vy, vz, mass, m_scalar, state, periodic,
                                         box, i, j, h, h_all, c.a, dt, xsec, s0, w0, model);
        double u = oref_uniform_decision(seed, step, id[i], id[j]);
        fl[dc] = (uint8_t)((fl[dc] & ~F_FLAGT) | (fabs(P - u) < band ? F_FLAGT : 0));
        if (!(u < P)) continue;
        do_kick(ph, i, j, mass, m_scalar, vx, vy, vz, state, id);
        int32_t dd = 1 + (depth[i] > depth[j] ? depth[i] : depth[j]);
        depth[i] = depth[j] = dd;
        if (dd > st->n_passes) st->n_passes = dd;
        st->n_events++;
        if (cand_info) cand_info[c.c] |= OREF_CAND_SCATTER | ((uint32_t)dd << 8);
        /* later turns touching i or j now see kicked velocities */
        int32_t pp[2] = {i, j};
        for (int q = 0; q < 2; ++q) {
            int32_t p = pp[q];
            int64_t ap = a_of[p];
            int64_t lo = ap >= 0 ? row_off[ap] : 0, hi = ap >= 0 ? row_off[ap + 1] : 0;
            for (int pass = 0; pass < 2; ++pass) {
                int64_t b0 = pass == 0 ? lo : rstart[p], b1 = pass == 0 ? hi : rstart[p + 1];
                for (int64_t t = b0; t < b1; ++t) {
                    int64_t d = pass == 0 ? t : rlist[t];
                    if (fl[d] & F_QUEUED) continue;
                    int64_t ad = pass == 0 ? ap : row_of(row_off, n_active, d);
                    cand_ord_t e;
                    TURN_OF(d, ad, e);
                    if (cand_ord_cmp(&e, &c) <= 0) continue;     /* its turn has passed */
                    fl[d] |= F_QUEUED;
                    if (heap_push(&hp, e)) { rc = OREF_E_NOMEM; goto done; }
                }
            }
        }
    }
#undef TURN_OF
    /* flagged at the turn: the visited turns' own evaluation, else the
     * step-start one (which is what the turn would have computed) */
    for (int64_t a = 0; a < n_active; ++a)
        for (int64_t d = row_off[a]; d < row_off[a + 1]; ++d) {
            int64_t ci = a * (int64_t)stride + (d - row_off[a]);
            int f = (fl[d] & F_QUEUED) ? (fl[d] & F_FLAGT) != 0 : (fl[d] & F_FLAG0) != 0;
            if (cand_info && (fl[d] & F_ACC0)) cand_info[ci] |= OREF_CAND_ACCEPT0;
            if (f) {
                st->n_flagged++;
                if (cand_info) cand_info[ci] |= OREF_CAND_FLAGGED;
            }
        }
done:
    free(hp.e); free(depth); free(rlist); free(rstart); free(a_of); free(fl);
    return rc;
}

static int scatter_core(int64_t n, const double *x, const double *y, const double *z,
                        double *vx, double *vy, double *vz, const double *mass, double m_scalar,
                        const uint32_t *id, uint8_t *state, int periodic, double box,
                        int64_t n_active, const int32_t *active, int stride, const int32_t *count,
                        const int32_t *ngb, const double *h, const double *h_all, const double *dt,
                        int xsec, double s0, double w0, int model, double eps, double delta,
                        uint64_t seed, uint32_t step, double band,
                        uint32_t *cand_info, oref_stats *stats)
{
    phys_t ph = {xsec, s0, w0, model, eps, delta, seed, step};
    oref_stats st; memset(&st, 0, sizeof st);
    if (cand_info) memset(cand_info, 0, (size_t)(n_active * (int64_t)stride) * sizeof(uint32_t));

    /* row a's candidates start at row_off[a] in the ordering array */
    int64_t *row_off = (int64_t *)malloc((size_t)(n_active + 1) * sizeof(int64_t));
    if (!row_off) return OREF_E_NOMEM;
    row_off[0] = 0;
    for (int64_t a = 0; a < n_active; ++a) {
        int len = stride;
        if (count && count[a] < len) len = count[a];
        row_off[a + 1] = row_off[a] + len;
    }
    const int64_t n_cand = row_off[n_active];
    st.n_cand = n_cand;
    if (oref_turn_mode == 1) {
        int rc = scatter_events(n, x, y, z, vx, vy, vz, mass, m_scalar, id, state, periodic, box,
                                n_active, active, stride, ngb, h, h_all, dt, &ph, band, row_off,
                                n_cand, cand_info, &st);
        free(row_off);
        if (stats) *stats = st;
        return rc;
    }
    cand_ord_t *ord = (cand_ord_t *)malloc((size_t)(n_cand > 0 ? n_cand : 1) * sizeof(cand_ord_t));
    int32_t *depth = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!ord || !depth) { free(ord); free(depth); free(row_off); return OREF_E_NOMEM; }

    /* the step-start evaluation (diagnostics only) and every candidate's key */
    double max_p = 0.0;
    int64_t n_ge1 = 0, n_acc0 = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : max_p) reduction(+ : n_ge1, n_acc0)
    for (int64_t a = 0; a < n_active; ++a) {
        int32_t i = active[a];
        int len = (int)(row_off[a + 1] - row_off[a]);
        for (int s = 0; s < len; ++s) {
            int64_t ci = a * (int64_t)stride + s;
            int32_t j = ngb[ci];
            double P = candidate_probability(x, y, z, vx, vy, vz, mass, m_scalar, state, periodic,
                                             box, i, j, h, h_all, a, dt, xsec, s0, w0, model);
            double u = oref_uniform_decision(seed, step, id[i], id[j]);
            if (P > max_p) max_p = P;
            if (P >= 1.0) n_ge1++;
            if (u < P) {
                n_acc0++;
                if (cand_info) cand_info[ci] |= OREF_CAND_ACCEPT0;
            }
            uint32_t xr[4];
            pair_draw(seed, step, id[i], id[j], PURPOSE_PRIORITY, xr);
            cand_ord_t e = {direction_word(xr, id[i] < id[j]), id[i], id[j], ci, a};
            ord[row_off[a] + s] = e;
        }
    }
    free(row_off);
    st.max_p = max_p;
    st.n_p_ge_1 = n_ge1;
    st.n_accept0 = n_acc0;

    /* every candidate at its turn, with the velocities as they are then */
    qsort(ord, (size_t)n_cand, sizeof(cand_ord_t), cand_ord_cmp);
    for (int64_t t = 0; t < n_cand; ++t) {
        const cand_ord_t *c = &ord[t];
        int32_t i = active[c->a], j = ngb[c->c];
        double P = candidate_probability(x, y, z, vx, vy, vz, mass, m_scalar, state, periodic,
                                         box, i, j, h, h_all, c->a, dt, xsec, s0, w0, model);
        double u = oref_uniform_decision(seed, step, id[i], id[j]);
        if (fabs(P - u) < band) {
            st.n_flagged++;
            if (cand_info) cand_info[c->c] |= OREF_CAND_FLAGGED;
        }
        if (u < P) {
            do_kick(&ph, i, j, mass, m_scalar, vx, vy, vz, state, id);
            int32_t d = 1 + (depth[i] > depth[j] ? depth[i] : depth[j]);
            depth[i] = depth[j] = d;
            if (d > st.n_passes) st.n_passes = d;
            st.n_events++;
            if (cand_info) cand_info[c->c] |= OREF_CAND_SCATTER | ((uint32_t)d << 8);
        }
    }
    free(depth);
    free(ord);
    if (stats) *stats = st;
    return OREF_OK;
}

int oref_scatter_step(int64_t n, const double *x, const double *y, const double *z,
                      double *vx, double *vy, double *vz, const double *mass, double m_scalar,
                      const uint32_t *id, uint8_t *state, int periodic, double box,
                      int64_t n_active, const int32_t *active, int k,
                      const int32_t *ngb, const double *h, const double *dt,
                      int xsec, double s0, double w0, int model, double eps, double delta,
                      uint64_t seed, uint32_t step, double band,
                      uint32_t *cand_info, oref_stats *stats)
{
    if (n < k + 2 || k < 1) return OREF_E_INVAL;
    return scatter_core(n, x, y, z, vx, vy, vz, mass, m_scalar, id, state, periodic, box,
                        n_active, active, k, NULL, ngb, h, NULL, dt, xsec, s0, w0, model, eps,
                        delta, seed, step, band, cand_info, stats);
}

/* ------------------------------------------------------------------------ */
/* Per-pair timestep (Eq. sidm_timestep), with the current velocities:        */
/* dt_i = C 2 / (m_DM W(0,h_i) max_j w_ij sigma(w_ij)/m); +inf if the max is 0 */
/* ------------------------------------------------------------------------ */
int oref_pair_timestep(int64_t n, const double *vx, const double *vy, const double *vz,
                       const double *mass, double m_scalar,
                       int64_t n_active, const int32_t *active, int k,
                       const int32_t *ngb, const double *h,
                       int xsec, double s0, double w0, double c_sidm, double *dt_out)
{
    if (n < k + 2 || k < 1) return OREF_E_INVAL;
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n_active; ++a) {
        int32_t i = active[a];
        double rmax = 0.0;
        for (int s = 0; s < k; ++s) {
            int32_t j = ngb[a * k + s];
            double w = oref_vel * rel_speed(vx[i], vy[i], vz[i], vx[j], vy[j], vz[j]);
            double ws = w * oref_sigma(w, xsec, s0, w0);
            if (ws > rmax) rmax = ws;
        }
        double mi = mass ? mass[i] : m_scalar;
        double W0 = oref_kernel(0.0, oref_len * h[a]);
        dt_out[a] = rmax > 0.0 ? (2.0 * c_sidm) / ((mi * W0) * rmax) : INFINITY;
    }
    return OREF_OK;
}

/* pair kick exposed for the conservation tests */
void oref_kick_pair(int32_t i, int32_t j, const double *mass, double m_scalar,
                    double *vx, double *vy, double *vz, uint8_t *state, const uint32_t *id,
                    int model, double eps, double delta, uint64_t seed, uint32_t step)
{
    phys_t ph = {0, 0.0, 1.0, model, eps, delta, seed, step};
    do_kick(&ph, i, j, mass, m_scalar, vx, vy, vz, state, id);
}

/* ======================================================================== */
/* Kernel-overlap estimator (Eq. kernelOverlap; the appendix comparing it   */
/* with the one-sided spline)                                                */
/* ======================================================================== */
#define OREF_OVL_NA 64      /* alpha = a / (2 NA), a = 0..NA, over [0, 1/2] */
#define OREF_OVL_NR 256     /* rho = b / NR, b = 0..NR, over [0, 1]          */

/* n-point Gauss-Legendre nodes and weights on [-1, 1]: the roots of P_n by
 * Newton's method from the usual cosine guesses, P_n and P_{n-1} from the
 * three-term recurrence, weight 2 / ((1 - x^2) P_n'(x)^2) */
static void gauss_legendre(int n, double *xn, double *wn)
{
    for (int i = 0; i < n; ++i) {
        double t = cos(OREF_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double step = p1 / dp;
            t -= step;
            if (fabs(step) < 1e-17) break;
        }
        xn[i] = t;
        wn[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

static double gl4x[4], gl4w[4], gl8x[8], gl8w[8];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    gauss_legendre(4, gl4x, gl4w);
    gauss_legendre(8, gl8x, gl8w);
    gl_ready = 1;
}

/* int_a^b t W(t, hj) dt; the integrand is a polynomial of degree 4 on each
 * side of hj/2, so a 4-point rule per piece is exact */
static double inner_integral(double a, double b, double hj)
{
    if (b > hj) b = hj;
    if (!(a < b)) return 0.0;
    double cut[3] = {a, b, b};
    int nc = 2;
    if (a < 0.5 * hj && 0.5 * hj < b) { cut[1] = 0.5 * hj; cut[2] = b; nc = 3; }
    double sum = 0.0;
    for (int p = 0; p + 1 < nc; ++p) {
        double mid = 0.5 * (cut[p] + cut[p + 1]), half = 0.5 * (cut[p + 1] - cut[p]);
        for (int q = 0; q < 4; ++q) {
            double t = mid + half * gl4x[q];
            sum += half * gl4w[q] * (t * oref_kernel(t, hj));
        }
    }
    return sum;
}

/* sort a short array in place */
static void sort_small(double *v, int n)
{
    for (int a = 1; a < n; ++a) {
        double t = v[a];
        int b = a - 1;
        while (b >= 0 && v[b] > t) { v[b + 1] = v[b]; --b; }
        v[b + 1] = t;
    }
}

/*
 * g(hi, hj, r) = int W(|x - x_i|, hi) W(|x - x_j|, hj) d^3x with r = |x_i - x_j|
 * (Eq. kernelOverlap), evaluated without tables.  In spherical coordinates
 * about x_i, with s = |x - x_i| and t = |x - x_j|, the volume element is
 * (2 pi / r) s t ds dt, so for r > 0
 *     g = (2 pi / r) int_0^hi s W(s, hi) [ int_{|r-s|}^{r+s} t W(t, hj) dt ] ds,
 * and g(r = 0) = 4 pi int s^2 W(s, hi) W(s, hj) ds.  The outer integrand is a
 * piecewise polynomial of degree <= 9 whose pieces end where s, |r - s| or
 * r + s meet hi/2, hj/2 or hj; an 8-point rule per piece is exact.
 */
double oref_overlap_exact(double hi, double hj, double r)
{
    gl_init();
    if (!(hi > 0.0) || !(hj > 0.0) || !(r < hi + hj)) return 0.0;
    if (r == 0.0) {
        double top = hi < hj ? hi : hj;
        double cut[4] = {0.0, 0.5 * hi, 0.5 * hj, top};
        sort_small(cut, 4);
        double sum = 0.0;
        for (int p = 0; p < 3; ++p) {
            double lo = cut[p], hi2 = cut[p + 1] < top ? cut[p + 1] : top;
            if (!(hi2 > lo)) continue;
            double mid = 0.5 * (lo + hi2), half = 0.5 * (hi2 - lo);
            for (int q = 0; q < 8; ++q) {
                double s = mid + half * gl8x[q];
                sum += half * gl8w[q] * ((s * s) * oref_kernel(s, hi) * oref_kernel(s, hj));
            }
        }
        return 4.0 * OREF_PI * sum;
    }
    double cand[10] = {0.0, hi, 0.5 * hi, r, r - 0.5 * hj, r + 0.5 * hj, r - hj, r + hj,
                       0.5 * hj - r, hj - r};
    double cut[10];
    int nc = 0;
    for (int c = 0; c < 10; ++c)
        if (cand[c] >= 0.0 && cand[c] <= hi) cut[nc++] = cand[c];
    sort_small(cut, nc);
    double sum = 0.0;
    for (int p = 0; p + 1 < nc; ++p) {
        if (!(cut[p + 1] > cut[p])) continue;
        double mid = 0.5 * (cut[p] + cut[p + 1]), half = 0.5 * (cut[p + 1] - cut[p]);
        for (int q = 0; q < 8; ++q) {
            double s = mid + half * gl8x[q];
            double in = inner_integral(fabs(r - s), r + s, hj);
            sum += half * gl8w[q] * (s * oref_kernel(s, hi) * in);
        }
    }
    return (2.0 * OREF_PI / r) * sum;
}

/* Table of the dimensionless overlap ghat(alpha, rho) = H^3 g(alpha H,
 * (1 - alpha) H, rho H), H = h_i + h_j, which by symmetry needs only
 * alpha = min(h_i, h_j) / H in [0, 1/2].  alpha = 0 is the limit of a point
 * partner, g = W(r, H). */
static double ovl_tab[(OREF_OVL_NA + 1) * (OREF_OVL_NR + 1)];
static int ovl_ready = 0;

static void ovl_build(void)
{
    if (ovl_ready) return;
    for (int a = 0; a <= OREF_OVL_NA; ++a) {
        double al = (double)a / (2.0 * OREF_OVL_NA);
        for (int b = 0; b <= OREF_OVL_NR; ++b) {
            double rho = (double)b / OREF_OVL_NR;
            ovl_tab[a * (OREF_OVL_NR + 1) + b] =
                a == 0 ? oref_kernel(rho, 1.0) : oref_overlap_exact(al, 1.0 - al, rho);
        }
    }
    ovl_ready = 1;
}

void oref_overlap_table(double *out)
{
    ovl_build();
    memcpy(out, ovl_tab, sizeof ovl_tab);
}

/* g_ij of the estimator: the table, bilinear in (alpha, rho), over H^3;
 * zero for r >= h_i + h_j */
double oref_overlap_g(double hi, double hj, double r)
{
    ovl_build();
    double H = hi + hj;
    double al = (hi < hj ? hi : hj) / H;
    double rho = r / H;
    if (!(rho < 1.0)) return 0.0;
    double fa = al * (2.0 * OREF_OVL_NA), fr = rho * OREF_OVL_NR;
    int ia = (int)fa, ir = (int)fr;
    if (ia > OREF_OVL_NA - 1) ia = OREF_OVL_NA - 1;
    if (ir > OREF_OVL_NR - 1) ir = OREF_OVL_NR - 1;
    double ta = fa - ia, tr = fr - ir;
    const double *t0 = ovl_tab + ia * (OREF_OVL_NR + 1) + ir;
    const double *t1 = t0 + (OREF_OVL_NR + 1);
    double g0 = t0[0] + tr * (t0[1] - t0[0]);
    double g1 = t1[0] + tr * (t1[1] - t1[0]);
    return (g0 + ta * (g1 - g0)) / ((H * H) * H);
}

/*
 * Partners of the overlap estimator by brute force: every j != i with
 * r_ij < h_i + h_j (tested as r^2 < (h_i + h_j)^2), in increasing j.  Row a
 * holds up to max_ngb of them, padded with -1; count[a] is the full number.
 * Returns the largest count.
 */
int64_t oref_find_overlap(int64_t n, const double *x, const double *y, const double *z,
                          int periodic, double box, const double *h_all, int64_t n_active,
                          const int32_t *active, int32_t max_ngb, int32_t *ngb, int32_t *count)
{
    int64_t most = 0;
    for (int64_t a = 0; a < n_active; ++a) {
        int32_t i = active[a];
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = oref_r2(x[i], y[i], z[i], x[j], y[j], z[j], periodic, box);
            double s = h_all[i] + h_all[j];
            if (r2 < s * s) {
                if (c < max_ngb) ngb[a * (int64_t)max_ngb + c] = (int32_t)j;
                c++;
            }
        }
        for (int32_t t = c; t < max_ngb; ++t) ngb[a * (int64_t)max_ngb + t] = -1;
        count[a] = c;
        if (c > most) most = c;
    }
    return most;
}

int oref_scatter_overlap(int64_t n, const double *x, const double *y, const double *z,
                         double *vx, double *vy, double *vz, const double *mass, double m_scalar,
                         const uint32_t *id, uint8_t *state, int periodic, double box,
                         const double *h_all, int64_t n_active, const int32_t *active,
                         int32_t max_ngb, const int32_t *ngb, const int32_t *count,
                         const double *dt, int xsec, double s0, double w0, int model, double eps,
                         double delta, uint64_t seed, uint32_t step, double band,
                         uint32_t *cand_info, oref_stats *stats)
{
    if (max_ngb < 1 || !h_all || !count) return OREF_E_INVAL;
    return scatter_core(n, x, y, z, vx, vy, vz, mass, m_scalar, id, state, periodic, box,
                        n_active, active, max_ngb, count, ngb, NULL, h_all, dt, xsec, s0, w0,
                        model, eps, delta, seed, step, band, cand_info, stats);
}

/*
 * Per-pair timestep with the overlap estimator: the bound of Eq. sidm_timestep
 * with the kernel's centre value W(0, h_i) replaced by the pair's overlap at
 * zero separation, g_ij(0) (the largest value g_ij takes):
 *     dt_i = C_SIDM * 2 / (m_i max_j [g_ij(0) w_ij sigma(w_ij)/m]),
 * so that P(i|j) <= C_SIDM for every partner while the velocities hold.
 */
int oref_pair_timestep_overlap(int64_t n, const double *vx, const double *vy, const double *vz,
                               const double *mass, double m_scalar, const double *h_all,
                               int64_t n_active, const int32_t *active, int32_t max_ngb,
                               const int32_t *ngb, const int32_t *count, int xsec, double s0,
                               double w0, double c_sidm, double *dt_out)
{
    (void)n;
    for (int64_t a = 0; a < n_active; ++a) {
        int32_t i = active[a];
        int len = count[a] < max_ngb ? count[a] : max_ngb;
        double qmax = 0.0;
        for (int s = 0; s < len; ++s) {
            int32_t j = ngb[a * (int64_t)max_ngb + s];
            double w = oref_vel * rel_speed(vx[i], vy[i], vz[i], vx[j], vy[j], vz[j]);
            double q = oref_overlap_g(oref_len * h_all[i], oref_len * h_all[j], 0.0) *
                       (w * oref_sigma(w, xsec, s0, w0));
            if (q > qmax) qmax = q;
        }
        double mi = mass ? mass[i] : m_scalar;
        dt_out[a] = qmax > 0.0 ? (2.0 * c_sidm) / (mi * qmax) : INFINITY;
    }
    return OREF_OK;
}
