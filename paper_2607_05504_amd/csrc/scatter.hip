// Scattering step of the active particles (paper sec. 4.1, 4.5) and the
// per-pair timestep bound (sec. 4.4, Eq. sidm_timestep).
//
// Semantics (sec. 4.5, immediate update): every directed candidate (i|j)
// takes one turn, in increasing key (priority, id_i, id_j); at its turn P is
// computed with the velocities of that moment and it scatters iff u < P.
// The step reproduces that serial order exactly, in parallel:
//
//  k_eval      one thread per candidate: P(i|j) = 1/2 m_j sigma(w)/m w
//              W(r_ij, h_i) dt_i (Eqs. rate, oneSided, probabilityScatter)
//              with the step-start velocities, the Philox decision draw, and
//              compaction of the accepted candidates into the list of
//              candidates whose turns are replayed ("listed").
//  passes      the listed candidates take their turns in key order: a pass
//              lets every candidate that holds the smallest key at both of
//              its particles evaluate P with the current velocities and kick
//              (these winners form a matching, so each particle takes at most
//              one turn per pass); the others wait.  Claims are 64-bit
//              integer atomicMin (priority, then the ID pair).  Each turn
//              appends a record to both particles' histories (key, velocity
//              before the turn, kicked or not).
//  k_check     one thread per candidate: a candidate touching a particle with
//              a history is evaluated at its turn, with the velocities the
//              histories give at its key.  A candidate that is not listed but
//              accepts there would have changed the step: it is listed.
//              If no candidate is, the replayed turns are the serial order
//              (every unlisted candidate rejects at its turn, so it changes
//              nothing), and the check's counts are the step's.  On long
//              steps the first check also writes a summary of each block of
//              1024 candidates (the index buckets its particles lie in), and
//              a later check scans only the blocks with a bucket holding a
//              particle of D.
//  k_reround   one workgroup: the turns that a newly listed candidate can
//              affect (later turns of its particles, closed under sharing a
//              particle) are rewound -- those particles' velocities restored
//              from their histories -- and taken again with the new ones;
//              then the next check.  A bounded number of rounds run as grid
//              launches, the rest in one workgroup (k_tail) until no
//              candidate is newly listed.
//  k_timestep  dt_i = 2 C_SIDM / (m_i W(0, h_i) max_j w_ij sigma(w_ij)/m).
#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMultiPasses = 4;        // passes run as grid-wide kernels
constexpr int kEvalGrid = 6 * 256;     // evaluation workgroups at least (fewer were slower)
constexpr int kFinisherMax = 256;      // shorter lists go to the one-workgroup finisher

// control words: [0..1] pass list counts, [2] completed passes, [3] hand-off
// flag, [4] listed candidates, [5] turn-record pairs ever used (x2), [6]
// first candidate listed since the last replay, [7] done (no candidate newly
// listed), [8] free record pairs, [9] re-rounds run, [10] particles of D
// (in plist), [11] flagged candidates listed for the final count, [12] index
// buckets holding a particle of D
enum { CTL_COUNT0 = 0, CTL_COUNT1 = 1, CTL_PASS = 2, CTL_HANDOFF = 3, CTL_MEM = 4, CTL_REC = 5,
       CTL_NEWLO = 6, CTL_DONE = 7, CTL_FREE = 8, CTL_ROUNDS = 9, CTL_PL = 10, CTL_FLAG = 11,
       CTL_DBK = 12 };

struct StepArgs {
    // Morton-ordered snapshot
    const double *xs, *ys, *zs, *ms;
    double *vxs, *vys, *vzs;
    const uint32_t *ids;
    uint8_t *sts;
    const int32_t *perm, *inv;
    // caller arrays (write-back)
    double *vx, *vy, *vz;
    uint8_t *state;
    // step inputs
    const int32_t *tlist, *slot, *nt_dev;
    const int32_t *ngb;
    const double *h, *dt;
    uint32_t *cand_info;
    // resolution: listed candidates, pass lists, histories
    AccList M;
    int32_t *wl0, *wl1, *mmark, *plist, *head, *rfree;
    TurnRecords R;
    unsigned long long *tmin;
    uint32_t *dbits;
    uint32_t *bbits;         // bit per index bucket holding a particle of D
    int64_t nbw;             // its words for n particles
    int32_t *csum;           // row block summaries of the step's rows, or NULL
    int32_t *flist;
    int32_t *jsort;          // the step's rows in Morton order (sorted indices), or NULL
    const double4 *vaos;     // velocities as (vx, vy, vz, 0) records for the timestep's gathers, or NULL
    const double2 *erec;     // per particle (x, y), (z, vx), (vy, vz), (id bits, mass): the evaluation's gathers
    int recs, verify_rows;   // the row-wise evaluation uses erec; and checks the rows against ngb
    int32_t *ctl;
    unsigned long long *c1a, *c1b, *c2a, *c2b;
    DevStats *st;
    unsigned int *derr;
    int64_t n, cap_acc, cap_rec;
    double m_scalar, box, s0, w0, eps, delta, band;
    // mixed form: FP32 offsets from the leaf box centres, and the relative
    // |P - u| band inside which an FP32 decision is redone in FP64
    const float *xo, *yo, *zo;
    const double *nodes;
    double band_p;
    // tabulated cross-section (SIDM_XSEC_TABLE)
    const double *xt_w, *xt_s, *xt_lw;
    int xt_n;
    // candidate rows: stride entries a row (n_ngb for the one-sided
    // estimator); the overlap estimator's rows hold count[a] partners and
    // take g_ij from every particle's h (hsrt, Morton order) and the table
    int stride;
    const int32_t *cnt;
    const double *hsrt, *gtab;
    // stored -> physical factors of lengths and relative speeds (comoving
    // storage): W, g_ij, sigma, P, the two-state balance and dt are physical
    double lphys, vphys;
    uint64_t seed;
    uint32_t step;
    int k, periodic, xsec, model, has_mass;
};

__device__ __forceinline__ double sigma_of(const StepArgs &A, double w)
{
    if (A.xsec == SIDM_XSEC_TABLE) return xsec_table(w, A.xt_w, A.xt_lw, A.xt_s, A.xt_n);
    return xsec_sigma(w, A.xsec, A.s0, A.w0);
}

__device__ __forceinline__ double mass_of(const StepArgs &A, int32_t s)
{
    return A.has_mass ? A.ms[s] : A.m_scalar;
}

// Sorted index of the partner of candidate c = b * stride + s (target b in
// Morton order, caller row a, ci = a * stride + s): from the step's sorted
// rows when it has them, else through inv (-1 for an index out of range).
__device__ __forceinline__ int32_t partner(const StepArgs &A, int64_t c, int64_t ci)
{
    if (A.jsort) return A.jsort[c];
    const int32_t jc = A.ngb[ci];
    return (jc >= 0 && jc < A.n) ? A.inv[jc] : -1;
}

// Target of candidate c (rows of stride entries): a shift for a power-of-two
// stride (sh >= 0), else a 32-bit division while the candidates fit 31 bits.
__device__ __forceinline__ int64_t row_of_cand(int64_t c, int sh, int stride, int64_t total)
{
    if (sh >= 0) return c >> sh;
    return total < 0x7fffffff ? (int64_t)((uint32_t)c / (uint32_t)stride) : c / stride;
}
__device__ __forceinline__ int stride_shift(int stride)
{
    return (stride & (stride - 1)) == 0 ? __ffs(stride) - 1 : -1;
}

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// wave-aggregated counter increment; returns this lane's slot (valid lanes only)
__device__ __forceinline__ int64_t wave_append(int32_t *counter, bool on)
{
    uint64_t m = __ballot(on);
    if (!m) return -1;
    int leader = __ffsll((long long)m) - 1;
    int lane = wave_lane();
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    return on ? (int64_t)base + __popcll(m & lt) : -1;
}

__device__ __forceinline__ void wave_count(unsigned long long *ctr, bool on)
{
    uint64_t m = __ballot(on);
    if (m && wave_lane() == __ffsll((long long)m) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// ----------------------------------------------------------------------------
// Scatter models: outgoing/incoming relative-speed ratio eps and state changes
// (sec. 4.1: the centre-of-momentum kinetic energy changes by eps^2).
// ----------------------------------------------------------------------------
__device__ double scatter_eps(const StepArgs &A, double ma, double mb, double w, uint8_t sa,
                              uint8_t sb, uint32_t ida, uint32_t idb, uint32_t bit,
                              uint8_t &nsa, uint8_t &nsb)
{
    nsa = sa;
    nsb = sb;
    if (A.model == SIDM_MODEL_EPS) return A.eps;
    if (A.model != SIDM_MODEL_TWO_STATE) return 1.0;
    double M = ma + mb;
    double mu = (ma * mb) / M;
    bool a_lower = ida < idb;
    if (sa == 0 && sb == 0) {
        bool excite_a = (bit == 0) ? a_lower : !a_lower;
        double mp = excite_a ? ma : mb;
        double e2 = 1.0 - (2.0 * mp * A.delta) / ((mu * w) * w);
        if (!(e2 > 0.0)) return 1.0;
        if (excite_a) nsa = 1; else nsb = 1;
        return sqrt(e2);
    }
    bool deexcite_a = (sa && sb) ? ((bit == 0) ? a_lower : !a_lower) : (sa != 0);
    double mp = deexcite_a ? ma : mb;
    double e2 = 1.0 + (2.0 * mp * A.delta) / ((mu * w) * w);
    if (deexcite_a) nsa = 0; else nsb = 0;
    return sqrt(e2);
}

// Kick of the pair (i, j) in Morton order, centre-of-momentum frame, direction
// uniform on the sphere from the pair's direction draw.
// beam model: only pairs of different populations scatter
__device__ __forceinline__ bool pair_allowed(const StepArgs &A, int32_t i, int32_t j)
{
    return A.model != SIDM_MODEL_BEAM || A.sts[i] != A.sts[j];
}

// Fixed-target limit (beam model): the target (state 0) keeps its velocity;
// the beam particle's velocity relative to it turns to the drawn direction
// with unchanged speed (+e if the beam particle is i, -e if it is j: the
// limit of the centre-of-momentum kick for an infinitely heavy target).
__device__ void kick_beam(const StepArgs &A, int32_t i, int32_t j, double ex, double ey, double ez)
{
    const double vix = A.vxs[i], viy = A.vys[i], viz = A.vzs[i];
    const double vjx = A.vxs[j], vjy = A.vys[j], vjz = A.vzs[j];
    const double w = rel_speed(vix, viy, viz, vjx, vjy, vjz);
    if (A.sts[i] == 1) {
        const double nx = vjx + w * ex, ny = vjy + w * ey, nz = vjz + w * ez;
        A.vxs[i] = nx; A.vys[i] = ny; A.vzs[i] = nz;
        const int32_t oi = A.perm[i];
        A.vx[oi] = nx; A.vy[oi] = ny; A.vz[oi] = nz;
    } else {
        const double nx = vix - w * ex, ny = viy - w * ey, nz = viz - w * ez;
        A.vxs[j] = nx; A.vys[j] = ny; A.vzs[j] = nz;
        const int32_t oj = A.perm[j];
        A.vx[oj] = nx; A.vy[oj] = ny; A.vz[oj] = nz;
    }
}

__device__ void kick(const StepArgs &A, int32_t i, int32_t j)
{
    const uint32_t idi = A.ids[i], idj = A.ids[j];
    Philox4 x = pair_draw(A.seed, A.step, idi, idj,
                          idi < idj ? PURPOSE_DIR_LO_HI : PURPOSE_DIR_HI_LO);
    double u1 = unit_from_word((uint64_t)x.x1 << 32 | x.x0);
    double u2 = unit_from_word((uint64_t)x.x3 << 32 | x.x2);
    double cth = 2.0 * u1 - 1.0;
    double phi = 2.0 * SIDM_PI * u2;
    double s2 = 1.0 - cth * cth;
    double sth = sqrt(s2 > 0.0 ? s2 : 0.0);
    double ex = sth * cos(phi), ey = sth * sin(phi), ez = cth;
    if (A.model == SIDM_MODEL_BEAM) { kick_beam(A, i, j, ex, ey, ez); return; }

    const double mi = mass_of(A, i), mj = mass_of(A, j);
    const double vix = A.vxs[i], viy = A.vys[i], viz = A.vzs[i];
    const double vjx = A.vxs[j], vjy = A.vys[j], vjz = A.vzs[j];
    const double w = rel_speed(vix, viy, viz, vjx, vjy, vjz);
    uint8_t nsi, nsj;
    // the energy balance in physical speed; the kick itself in stored units
    double eps = scatter_eps(A, mi, mj, A.vphys * w, A.sts[i], A.sts[j], idi, idj, x.x0 & 1u,
                             nsi, nsj);
    double M = mi + mj;
    double vcx = (mi * vix + mj * vjx) / M;
    double vcy = (mi * viy + mj * vjy) / M;
    double vcz = (mi * viz + mj * vjz) / M;
    double c = (eps * w) / M;
    double ci = mj * c, cj = mi * c;
    double nix = vcx + ci * ex, niy = vcy + ci * ey, niz = vcz + ci * ez;
    double njx = vcx - cj * ex, njy = vcy - cj * ey, njz = vcz - cj * ez;
    A.vxs[i] = nix; A.vys[i] = niy; A.vzs[i] = niz;
    A.vxs[j] = njx; A.vys[j] = njy; A.vzs[j] = njz;
    const int32_t oi = A.perm[i], oj = A.perm[j];
    A.vx[oi] = nix; A.vy[oi] = niy; A.vz[oi] = niz;
    A.vx[oj] = njx; A.vy[oj] = njy; A.vz[oj] = njz;
    if (A.model == SIDM_MODEL_TWO_STATE) {
        A.sts[i] = nsi;
        A.sts[j] = nsj;
        if (A.state) { A.state[oi] = nsi; A.state[oj] = nsj; }
    }
}

// ----------------------------------------------------------------------------
// Evaluation 0: every candidate with the step-start velocities.  Accepted
// candidates are staged in LDS and appended to the list in bulk, and the
// statistics are reduced per workgroup, so global atomics stay per workgroup.
// A staged entry keeps only what cannot be looked up again (the candidate's
// index c = b * stride + s, its draw u and its W); the flush recomputes the
// rest, so that the buffer is small and more workgroups are resident.
// ----------------------------------------------------------------------------
constexpr int kStage = 512;                // staged accepted candidates per workgroup

struct StagedAcc {
    int64_t c[kStage];
    double u[kStage], W[kStage];
};

// the row-wise evaluation stages up to four candidates a thread a round
constexpr int kStageRows = 5 * 256;
struct StagedAccRows {
    int32_t c[kStageRows];
    double u[kStageRows], W[kStageRows];
};

template <class Stage>
__device__ void flush_staged(const StepArgs &A, Stage &S, int n, int32_t &base_s)
{
    if (threadIdx.x == 0) {
        base_s = atomicAdd(&A.ctl[CTL_MEM], n);
        atomicAdd(&A.ctl[CTL_COUNT0], n);     // the first pass list is every listed candidate
    }
    __syncthreads();
    const int64_t base = base_s;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int64_t pos = base + t;
        if (pos >= A.cap_acc) { atomicOr(A.derr, DERR_OVERFLOW); continue; }
        const int64_t c = S.c[t];
        const int64_t b = c / A.stride;
        const int s = (int)(c - b * A.stride);
        const int32_t a = A.slot[b], i = A.tlist[b];
        const int64_t ci = (int64_t)a * A.stride + s;
        const int32_t j = partner(A, c, ci);   // checked in range when it was evaluated
        const uint32_t idi = A.ids[i], idj = A.ids[j];
        const Philox4 xp = pair_draw(A.seed, A.step, idi, idj, PURPOSE_PRIORITY);
        A.M.i[pos] = i; A.M.j[pos] = j; A.M.cand[pos] = (int32_t)ci;
        A.M.u[pos] = S.u[t]; A.M.W[pos] = S.W[t]; A.M.dt[pos] = A.dt[a];
        A.M.prio[pos] = direction_word(xp, idi < idj);
        A.M.idpair[pos] = ((uint64_t)idi << 32) | idj;
        A.M.rec[pos] = -1;
        A.wl0[pos] = (int32_t)pos;
        A.c1a[i] = ~0ull; A.c1a[j] = ~0ull;
        A.c2a[i] = ~0ull; A.c2a[j] = ~0ull;
    }
    __syncthreads();
}

// FP32 forms of the kernel and cross-section (mixed form)
__device__ __forceinline__ float cubic_spline32(float r, float h)
{
    const float norm = 8.0f / ((float)SIDM_PI * ((h * h) * h));
    const float q = r / h;
    if (q <= 0.5f) {
        const float q2 = q * q;
        return norm * ((1.0f - 6.0f * q2) + 6.0f * (q2 * q));
    }
    if (q <= 1.0f) {
        const float t = 1.0f - q;
        return norm * (2.0f * ((t * t) * t));
    }
    return 0.0f;
}

__device__ __forceinline__ float xsec_sigma32(float w, int xsec, float s0, float w0)
{
    if (xsec == SIDM_XSEC_YUKAWA) {
        const float x = w / w0;
        const float d = 1.0f + x * x;
        return s0 / (d * d);
    }
    return s0;
}

// workgroup reduction of the evaluation's statistics, one atomic each
template <bool OVERLAP>
__device__ void eval_stats(const StepArgs &A, unsigned long long (&s_red)[4][6], unsigned long long maxp,
                           unsigned long long n_fl, unsigned long long n_ge1, unsigned long long n_acc,
                           unsigned long long n_rc, unsigned long long n_cd)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)maxp, off);
        maxp = o > maxp ? o : maxp;
        n_fl += (unsigned long long)__shfl_xor((long long)n_fl, off);
        n_ge1 += (unsigned long long)__shfl_xor((long long)n_ge1, off);
        n_acc += (unsigned long long)__shfl_xor((long long)n_acc, off);
        n_rc += (unsigned long long)__shfl_xor((long long)n_rc, off);
        n_cd += (unsigned long long)__shfl_xor((long long)n_cd, off);
    }
    const int w = threadIdx.x >> 6;
    if (wave_lane() == 0) {
        s_red[w][0] = maxp; s_red[w][1] = n_fl; s_red[w][2] = n_ge1; s_red[w][3] = n_acc; s_red[w][4] = n_rc;
        s_red[w][5] = n_cd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0, f = 0, g = 0, q = 0, rc = 0, cd = 0;
        for (int v = 0; v < kBlock / 64; ++v) {
            m = s_red[v][0] > m ? s_red[v][0] : m;
            f += s_red[v][1]; g += s_red[v][2]; q += s_red[v][3]; rc += s_red[v][4];
            cd += s_red[v][5];
        }
        if (OVERLAP && cd) atomicAdd(&A.st->n_cand, cd);
        if (rc) atomicAdd(&A.st->n_recheck, rc);
        if (m) atomicMax(&A.st->max_p_bits, m);
        if (f) atomicAdd(&A.st->n_flagged, f);
        if (g) atomicAdd(&A.st->n_p_ge_1, g);
        if (q) atomicAdd(&A.st->n_accept0, q);
    }
}

// W_CS(r, h) with the normalisation 8 / (pi h^3) given (computed as in
// cubic_spline, so the value is the same bit for bit)
__device__ __forceinline__ double spline_norm(double h)
{
    const double h3 = (h * h) * h;
    return 8.0 / (SIDM_PI * h3);
}
__device__ __forceinline__ double cubic_spline_n(double r, double h, double norm)
{
    const double q = r / h;
    if (q <= 0.5) {
        const double q2 = q * q;
        const double q3 = q2 * q;
        return norm * ((1.0 - 6.0 * q2) + 6.0 * q3);
    }
    if (q <= 1.0) {
        const double t = 1.0 - q;
        return norm * (2.0 * ((t * t) * t));
    }
    return 0.0;
}

// The evaluation's per-particle records (in the phase buffer, which the step
// does not otherwise use): a partner's data in one 64-byte line, the ID in
// the low and the caller index in the high half of the third word.
__global__ __launch_bounds__(kBlock) void k_eval_recs(StepArgs A, double2 *out)
{
    // a lane a 16-byte quarter of a record: consecutive lanes write
    // consecutive bytes
    const int64_t total = 4 * A.n;
    for (int64_t t = xcd_stride_block() * (int64_t)kBlock + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kBlock) {
        const int64_t q = t >> 2;
        const int part = (int)(t & 3);
        double2 v;
        if (part < 3) {
            const double *pa = part == 0 ? A.xs : part == 1 ? A.zs : A.vys;
            const double *pb = part == 0 ? A.ys : part == 1 ? A.vxs : A.vzs;
            v = make_double2(pa[q], pb[q]);
        } else {
            const uint64_t w = ((uint64_t)(uint32_t)A.perm[q] << 32) | A.ids[q];
            v = make_double2(__longlong_as_double((long long)w), mass_of(A, (int32_t)q));
        }
        out[t] = v;
    }
}

// k_eval of the FP64 one-sided form for rows of k = 2^sh >= 4 candidates: a
// lane takes four candidates of a row (k / 4 lanes a row), so that the
// target's data, its timestep and the kernel's normalisation are read and
// computed once for four.  Same arithmetic per candidate as k_eval.
template <bool PERIODIC, bool REC, bool VERIFY>
__global__ __launch_bounds__(kBlock) void k_eval_rows(StepArgs A)
{
    __shared__ StagedAccRows S;
    __shared__ int s_n;
    __shared__ int32_t s_base;
    __shared__ unsigned long long s_red[4][6];
    const int64_t nt = *A.nt_dev;
    const int sh = stride_shift(A.stride);    // >= 2 (checked by the launch)
    const int lsh = sh - 2;
    const int L = 1 << lsh;
    const int64_t lanes = nt << lsh;
    unsigned long long maxp = 0, n_fl = 0, n_ge1 = 0, n_acc = 0, n_rc = 0, n_cd = 0;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int64_t t0 = xcd_stride_block() * (int64_t)blockDim.x; t0 < lanes;
         t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        if (t < lanes) {
            const int64_t b = t >> lsh;
            const int l = (int)(t & (L - 1));
            const int32_t a = A.slot[b], i = A.tlist[b];
            const double dta = A.dt[a];
            const uint32_t idi = A.ids[i];
            const double xi = A.xs[i], yi = A.ys[i], zi = A.zs[i];
            const double vxi = A.vxs[i], vyi = A.vys[i], vzi = A.vzs[i];
            const double hp = A.lphys * A.h[a];
            const double norm = spline_norm(hp);
            // with records a lane takes four consecutive entries of the row
            // (one 16-byte load of the rows, and of ngb to check them), else
            // every L-th (the row's lanes read consecutive words)
            int32_t jj[4], jc[4];
            if constexpr (REC) {
                const int4 q = *(const int4 *)(A.jsort + (b << sh) + 4 * l);
                jj[0] = q.x; jj[1] = q.y; jj[2] = q.z; jj[3] = q.w;
                if constexpr (VERIFY) {
                    const int4 g = *(const int4 *)(A.ngb + (int64_t)a * A.stride + 4 * l);
                    jc[0] = g.x; jc[1] = g.y; jc[2] = g.z; jc[3] = g.w;
                }
            } else {
#pragma unroll
                for (int u4 = 0; u4 < 4; ++u4) {
                    const int sidx = l + u4 * L;
                    jj[u4] = partner(A, (b << sh) + sidx, (int64_t)a * A.stride + sidx);
                }
            }
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) {
                const int sidx = REC ? 4 * l + u4 : l + u4 * L;
                const int64_t c = (b << sh) + sidx;
                const int64_t ci = (int64_t)a * A.stride + sidx;
                int32_t j = jj[u4];
                n_cd += 1;
                // the partner's record (four 16-byte loads instead of eight
                // gathers), else its entries in the snapshot
                double2 r0, r1, r2, r3;
                if constexpr (VERIFY) {
                    // k_rows' check here: the row entry stands if the caller
                    // index in its record is the caller's ngb entry, else it
                    // is translated (and written back for the later kernels)
                    bool ok = j >= 0 && j < A.n;
                    if (ok) {
                        const double2 *R = A.erec + 4 * (int64_t)j;
                        r0 = R[0]; r1 = R[1]; r2 = R[2]; r3 = R[3];
                        ok = (int32_t)((uint64_t)__double_as_longlong(r3.x) >> 32) == jc[u4];
                    }
                    if (!ok) {
                        j = (jc[u4] >= 0 && jc[u4] < A.n) ? A.inv[jc[u4]] : -1;
                        if (j < 0) atomicOr(A.derr, DERR_INDEX);
                        A.jsort[c] = j;
                        if (j < 0) continue;
                        const double2 *R = A.erec + 4 * (int64_t)j;
                        r0 = R[0]; r1 = R[1]; r2 = R[2]; r3 = R[3];
                    }
                } else if constexpr (REC) {
                    if (j < 0) continue;                        // latched by k_rows
                    const double2 *R = A.erec + 4 * (int64_t)j;
                    r0 = R[0]; r1 = R[1]; r2 = R[2]; r3 = R[3];
                } else {
                    if (j < 0) {
                        if (!A.jsort) atomicOr(A.derr, DERR_INDEX);   // else latched by k_rows
                        continue;
                    }
                    r0 = make_double2(A.xs[j], A.ys[j]);
                    r1 = make_double2(A.zs[j], A.vxs[j]);
                    r2 = make_double2(A.vys[j], A.vzs[j]);
                    r3 = make_double2(__longlong_as_double((long long)A.ids[j]), mass_of(A, j));
                }
                const uint32_t idj = (uint32_t)__double_as_longlong(r3.x);
                const Philox4 x = pair_draw(A.seed, A.step, idi, idj, PURPOSE_DECIDE);
                const double u = unit_from_word(direction_word(x, idi < idj));
                const double r = A.lphys * sqrt(sep2<PERIODIC>(xi, yi, zi, r0.x, r0.y, r1.x, A.box));
                const double W = cubic_spline_n(r, hp, norm);
                const double w = A.vphys * rel_speed(vxi, vyi, vzi, r1.y, r2.x, r2.y);
                const double sig = sigma_of(A, w);
                double P = pair_prob(r3.y, sig, w, W, dta);
                if (!pair_allowed(A, i, j)) P = 0.0;
                const bool acc = u < P;
                const bool flagged = fabs(P - u) < A.band;
                n_fl += flagged;
                n_ge1 += P >= 1.0;
                n_acc += acc;
                const unsigned long long pb = (unsigned long long)__double_as_longlong(P);
                maxp = pb > maxp ? pb : maxp;
                if (A.cand_info)
                    A.cand_info[ci] = (acc ? SIDM_CAND_ACCEPT0 : 0u) | (flagged ? SIDM_CAND_FLAGGED : 0u);
                if (acc) {
                    const int q = atomicAdd(&s_n, 1);      // LDS; kStageRows >= 5 * blockDim
                    S.c[q] = (int32_t)c; S.u[q] = u; S.W[q] = W;
                }
            }
        }
        __syncthreads();
        const int n_st = s_n;
        // every wave has read s_n before any appends to it again
        __syncthreads();
        if (n_st > kStageRows - 4 * kBlock) {      // the next round might not fit
            flush_staged(A, S, n_st, s_base);
            if (threadIdx.x == 0) s_n = 0;
            __syncthreads();
        }
    }
    if (s_n > 0) flush_staged(A, S, s_n, s_base);
    eval_stats<false>(A, s_red, maxp, n_fl, n_ge1, n_acc, n_rc, n_cd);
}

template <bool PERIODIC, bool MIXED, bool OVERLAP>
__global__ __launch_bounds__(kBlock) void k_eval(StepArgs A)
{
    __shared__ StagedAcc S;
    __shared__ int s_n;
    __shared__ int32_t s_base;
    __shared__ unsigned long long s_red[4][6];
    const int64_t nt = *A.nt_dev;
    const int64_t total = nt * A.stride;
    const int sh = stride_shift(A.stride);
    unsigned long long maxp = 0, n_fl = 0, n_ge1 = 0, n_acc = 0, n_rc = 0, n_cd = 0;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int64_t c0 = xcd_stride_block() * (int64_t)blockDim.x; c0 < total;
         c0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = c0 + threadIdx.x;
        bool live = c < total;
        int64_t b = 0;
        int s = 0;
        int32_t a = 0;
        if (live) {
            b = row_of_cand(c, sh, A.stride, total);
            s = (int)(c - b * A.stride);
            a = A.slot[b];
            if (OVERLAP) live = s < A.cnt[a];
        }
        if (live) {
            const int32_t i = A.tlist[b];
            const int64_t ci = (int64_t)a * A.stride + s;
            const int32_t j = partner(A, c, ci);
            n_cd += 1;
            if (j < 0) {
                if (!A.jsort) atomicOr(A.derr, DERR_INDEX);   // else latched by k_rows
            } else {
                const double dta = A.dt[a];
                const uint32_t idi = A.ids[i], idj = A.ids[j];
                const Philox4 x = pair_draw(A.seed, A.step, idi, idj, PURPOSE_DECIDE);
                const double u = unit_from_word(direction_word(x, idi < idj));
                double P = 0.0, W = 0.0;
                bool exact = true;
                if constexpr (MIXED) {
                    // FP32: separation from the two leaves' box centres plus
                    // the particles' FP32 offsets; relative speed from the
                    // FP64 velocity difference rounded to FP32
                    const double *bi = A.nodes + (int64_t)(i / SIDM_LEAF) * 6;
                    const double *bj = A.nodes + (int64_t)(j / SIDM_LEAF) * 6;
                    const float bx = (float)A.box;
                    double cdx = box_centre(bj, 0) - box_centre(bi, 0);
                    double cdy = box_centre(bj, 1) - box_centre(bi, 1);
                    double cdz = box_centre(bj, 2) - box_centre(bi, 2);
                    if (PERIODIC) {
                        const double half = 0.5 * A.box;
                        cdx = cdx >= half ? cdx - A.box : (cdx < -half ? cdx + A.box : cdx);
                        cdy = cdy >= half ? cdy - A.box : (cdy < -half ? cdy + A.box : cdy);
                        cdz = cdz >= half ? cdz - A.box : (cdz < -half ? cdz + A.box : cdz);
                    }
                    const float oix = A.xo[i], oiy = A.yo[i], oiz = A.zo[i];
                    const float ojx = A.xo[j], ojy = A.yo[j], ojz = A.zo[j];
                    float dx = (float)cdx + (ojx - oix);
                    float dy = (float)cdy + (ojy - oiy);
                    float dz = (float)cdz + (ojz - oiz);
                    if (PERIODIC) { dx = wrap32(dx, bx); dy = wrap32(dy, bx); dz = wrap32(dz, bx); }
                    const float d2 = (dx * dx + dy * dy) + dz * dz;
                    // Each FP32 component of the separation errs by at most
                    // 3 2^-24 (|d| + |o_i| + |o_j|), d the separation and o
                    // the particles' offsets from their leaf centres.  The
                    // spline's slope is at most 1.5 W(0) / h, so while that sum
                    // stays below 12 h the error moves P by less than 5.6e-6 of
                    // its centre value (under 7e-6 with the other FP32
                    // roundings), inside band_p.  Particles far from their leaf
                    // centres (Morton neighbours spread over a jump of the
                    // curve) take the FP64 evaluation.  The sum's square is at
                    // most 3 (d^2 + o_i^2 + o_j^2).
                    const float o2 = ((oix * oix + oiy * oiy) + oiz * oiz) +
                                     ((ojx * ojx + ojy * ojy) + ojz * ojz);
                    const float hl = (float)A.h[a];
                    const bool far = !(3.0f * (d2 + o2) <= 143.0f * (hl * hl));
                    const float r32 = (float)A.lphys * sqrtf(d2);
                    const float h32 = (float)(A.lphys * A.h[a]);
                    const float vx = (float)(A.vxs[i] - A.vxs[j]), vy = (float)(A.vys[i] - A.vys[j]),
                                vz = (float)(A.vzs[i] - A.vzs[j]);
                    const float w32 = (float)A.vphys * sqrtf((vx * vx + vy * vy) + vz * vz);
                    const float s32 = A.xsec == SIDM_XSEC_TABLE
                                          ? (float)sigma_of(A, (double)w32)
                                          : xsec_sigma32(w32, A.xsec, (float)A.s0, (float)A.w0);
                    const float f = (((0.5f * (float)mass_of(A, j)) * s32) * w32) * (float)dta;
                    const float P32 = f * cubic_spline32(r32, h32);
                    // band on the scale of P at the kernel's centre value, so
                    // the absolute FP32 error of W near its support edge is covered
                    const float Pmax = f * (8.0f / ((float)SIDM_PI * ((h32 * h32) * h32)));
                    const double near = A.band_p * fmax((double)Pmax, u) + A.band;
                    P = pair_allowed(A, i, j) ? (double)P32 : 0.0;
                    exact = far || fabs(P - u) <= near;
                }
                if (exact) {
                    // physical separation, smoothing lengths and relative speed
                    const double r = A.lphys * sqrt(sep2<PERIODIC>(A.xs[i], A.ys[i], A.zs[i],
                                                                   A.xs[j], A.ys[j], A.zs[j], A.box));
                    W = OVERLAP ? overlap_g(A.gtab, A.lphys * A.hsrt[i], A.lphys * A.hsrt[j], r)
                                : cubic_spline(r, A.lphys * A.h[a]);
                    const double w = A.vphys * rel_speed(A.vxs[i], A.vys[i], A.vzs[i], A.vxs[j],
                                                         A.vys[j], A.vzs[j]);
                    const double sig = sigma_of(A, w);
                    P = pair_prob(mass_of(A, j), sig, w, W, dta);
                    if (!pair_allowed(A, i, j)) P = 0.0;
                    n_rc += MIXED;
                }
                const bool acc = u < P;
                const bool flagged = exact && fabs(P - u) < A.band;
                if (MIXED && acc && !exact) {
                    // accepted on the FP32 value: the passes need the FP64 W
                    const double r = A.lphys * sqrt(sep2<PERIODIC>(A.xs[i], A.ys[i], A.zs[i],
                                                                   A.xs[j], A.ys[j], A.zs[j], A.box));
                    W = cubic_spline(r, A.lphys * A.h[a]);
                }
                n_fl += flagged;
                n_ge1 += P >= 1.0;
                n_acc += acc;
                const unsigned long long pb = (unsigned long long)__double_as_longlong(P);
                maxp = pb > maxp ? pb : maxp;
                if (A.cand_info)
                    A.cand_info[ci] =
                        (acc ? SIDM_CAND_ACCEPT0 : 0u) | (flagged ? SIDM_CAND_FLAGGED : 0u);
                if (acc) {
                    const int t = atomicAdd(&s_n, 1);      // LDS; kStage >= 2 * blockDim
                    S.c[t] = c; S.u[t] = u; S.W[t] = W;
                }
            }
        }
        __syncthreads();
        const int n_st = s_n;
        // every wave has read s_n before any appends to it again
        __syncthreads();
        if (n_st > kStage - kBlock) {              // the next round might not fit
            flush_staged(A, S, n_st, s_base);
            if (threadIdx.x == 0) s_n = 0;
            __syncthreads();
        }
    }
    if (s_n > 0) flush_staged(A, S, s_n, s_base);
    eval_stats<OVERLAP>(A, s_red, maxp, n_fl, n_ge1, n_acc, n_rc, n_cd);
}

// ----------------------------------------------------------------------------
// Turns of the listed candidates.  Pass t reads work list t&1 (indices into
// the listed candidates) and claim buffers t&1.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int32_t *list_of(const StepArgs &A, int t) { return (t & 1) ? A.wl1 : A.wl0; }
__device__ __forceinline__ unsigned long long *claim1_of(const StepArgs &A, int t) { return (t & 1) ? A.c1b : A.c1a; }
__device__ __forceinline__ unsigned long long *claim2_of(const StepArgs &A, int t) { return (t & 1) ? A.c2b : A.c2a; }

__device__ __forceinline__ unsigned long long load_u64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_i32(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t list_count(const StepArgs &A, int t)
{
    int64_t c = A.ctl[(t & 1) ? CTL_COUNT1 : CTL_COUNT0];
    return c < A.cap_acc ? c : A.cap_acc;
}

__device__ __forceinline__ void claim1_entry(const StepArgs &A, int t, int64_t e)
{
    const int32_t m = list_of(A, t)[e];
    unsigned long long *c1 = claim1_of(A, t);
    const unsigned long long pr = A.M.prio[m];
    atomicMin(&c1[A.M.i[m]], pr);
    atomicMin(&c1[A.M.j[m]], pr);
}

__device__ __forceinline__ void claim2_entry(const StepArgs &A, int t, int64_t e)
{
    const int32_t m = list_of(A, t)[e];
    const unsigned long long *c1 = claim1_of(A, t);
    unsigned long long *c2 = claim2_of(A, t);
    const unsigned long long pr = A.M.prio[m], ip = A.M.idpair[m];
    const int32_t i = A.M.i[m], j = A.M.j[m];
    if (load_u64(&c1[i]) == pr) atomicMin(&c2[i], ip);
    if (load_u64(&c1[j]) == pr) atomicMin(&c2[j], ip);
}

__device__ __forceinline__ void put_record(const StepArgs &A, int32_t r, int32_t p, uint64_t pr,
                                           uint64_t ip, int32_t m, int32_t prev, uint32_t info)
{
    A.R.prio[r] = pr; A.R.idpair[r] = ip;
    A.R.vx[r] = A.vxs[p]; A.R.vy[r] = A.vys[p]; A.R.vz[r] = A.vzs[p];
    A.R.mem[r] = m; A.R.prev[r] = prev; A.R.part[r] = p;
    A.R.info[r] = info | ((uint32_t)A.sts[p] << 1);
}

// The turn of listed candidate m = (i|j): P with the current velocities, a
// record of the turn in both particles' histories, and the kick if u < P.
// Called only for a pass winner, so no other thread touches i or j.
__device__ void take_turn(const StepArgs &A, int32_t m)
{
    const int32_t i = A.M.i[m], j = A.M.j[m];
    const double w = A.vphys * rel_speed(A.vxs[i], A.vys[i], A.vzs[i], A.vxs[j], A.vys[j], A.vzs[j]);
    const double sig = sigma_of(A, w);
    const double P = pair_allowed(A, i, j) ? pair_prob(mass_of(A, j), sig, w, A.M.W[m], A.M.dt[m]) : 0.0;
    const bool hit = A.M.u[m] < P;
    // a record pair (r at i, r + 1 at j): one a rewind freed, else a new one
    int32_t r = -1;
    if (load_i32(&A.ctl[CTL_FREE]) > 0) {
        const int32_t f = atomicSub(&A.ctl[CTL_FREE], 1);
        if (f > 0) r = 2 * A.rfree[f - 1];
    }
    if (r < 0) r = atomicAdd(&A.ctl[CTL_REC], 2);
    if ((int64_t)r + 2 <= A.cap_rec) {
        const int32_t hi = A.head[i], hj = A.head[j];
        const uint32_t di = hi >= 0 ? A.R.info[hi] >> 8 : 0u, dj = hj >= 0 ? A.R.info[hj] >> 8 : 0u;
        const uint32_t d = 1u + (di > dj ? di : dj);     // depth of this kick
        const uint64_t pr = A.M.prio[m], ip = A.M.idpair[m];
        put_record(A, r, i, pr, ip, m, hi, hit ? (1u | (d << 8)) : (di << 8));
        put_record(A, r + 1, j, pr, ip, m, hj, hit ? (1u | (d << 8)) : (dj << 8));
        A.head[i] = r;
        A.head[j] = r + 1;
        A.M.rec[m] = r;
    } else {
        atomicOr(A.derr, DERR_HISTORY);
    }
    if (hit) kick(A, i, j);
}

// returns true if the entry took its turn (a winner) this pass
__device__ bool resolve_entry(const StepArgs &A, int t, int64_t e, int32_t *next_count)
{
    const int32_t m = list_of(A, t)[e];
    const unsigned long long *c1 = claim1_of(A, t), *c2 = claim2_of(A, t);
    const int32_t i = A.M.i[m], j = A.M.j[m];
    const unsigned long long pr = A.M.prio[m], ip = A.M.idpair[m];
    const bool win = load_u64(&c1[i]) == pr && load_u64(&c1[j]) == pr &&
                     load_u64(&c2[i]) == ip && load_u64(&c2[j]) == ip;
    if (win) {
        take_turn(A, m);
        return true;
    }
    // carry over to the next pass, and clear the claims it will use
    const int32_t pos = atomicAdd(next_count, 1);
    list_of(A, t + 1)[pos] = m;
    unsigned long long *n1 = claim1_of(A, t + 1), *n2 = claim2_of(A, t + 1);
    n1[i] = ~0ull; n1[j] = ~0ull;
    n2[i] = ~0ull; n2[j] = ~0ull;
    return false;
}

// a grid pass runs only while no hand-off happened and the list is long
__device__ __forceinline__ bool grid_pass_active(const StepArgs &A, int t)
{
    if (A.ctl[CTL_HANDOFF]) return false;
    return list_count(A, t) > kFinisherMax;
}

__global__ __launch_bounds__(kBlock) void k_claim1(StepArgs A, int t)
{
    if (!grid_pass_active(A, t)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl[CTL_HANDOFF] = 1;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl[((t + 1) & 1) ? CTL_COUNT1 : CTL_COUNT0] = 0;
    const int64_t cnt = list_count(A, t);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * blockDim.x)
        claim1_entry(A, t, e);
}

__global__ __launch_bounds__(kBlock) void k_claim2(StepArgs A, int t)
{
    if (A.ctl[CTL_HANDOFF]) return;
    const int64_t cnt = list_count(A, t);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * blockDim.x)
        claim2_entry(A, t, e);
}

__global__ __launch_bounds__(kBlock) void k_resolve(StepArgs A, int t)
{
    if (A.ctl[CTL_HANDOFF]) return;
    const int64_t cnt = list_count(A, t);
    int32_t *next = &A.ctl[((t + 1) & 1) ? CTL_COUNT1 : CTL_COUNT0];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * blockDim.x)
        resolve_entry(A, t, e, next);
    if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl[CTL_PASS] = t + 1;
}

__device__ __forceinline__ void wg_sync()
{
    __threadfence_block();
    __syncthreads();
}

// Passes of one workgroup over work list t0&1 holding cnt0 entries, until
// every entry has taken its turn.
struct PassShared { int64_t cnt; int t; };

__device__ void wg_passes(const StepArgs &A, int t0, int64_t cnt0, PassShared &S)
{
    if (threadIdx.x == 0) { S.t = t0; S.cnt = cnt0; }
    __syncthreads();
    while (S.cnt > 0) {
        const int t = S.t;
        const int64_t cnt = S.cnt;
        int32_t *next = &A.ctl[((t + 1) & 1) ? CTL_COUNT1 : CTL_COUNT0];
        if (threadIdx.x == 0) *next = 0;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) claim1_entry(A, t, e);
        wg_sync();
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) claim2_entry(A, t, e);
        wg_sync();
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) resolve_entry(A, t, e, next);
        wg_sync();
        if (threadIdx.x == 0) {
            S.t = t + 1;
            int64_t nc = load_i32(next);
            if (nc >= cnt) {            // no winner: the smallest key always wins
                atomicOr(A.derr, DERR_STALL);
                nc = 0;
            }
            S.cnt = nc;
        }
        __syncthreads();
    }
}

// D, the particles whose history changed since the last check, is marked by
// tmin != ~0 and by a bit per sorted index, which the check's scan tests.
__device__ __forceinline__ void set_dbit(const StepArgs &A, int32_t p)
{
    atomicOr(&A.dbits[p >> 5], 1u << (p & 31));
}
__device__ __forceinline__ void clear_dbit(const StepArgs &A, int32_t p)
{
    atomicAnd(&A.dbits[p >> 5], ~(1u << (p & 31)));
}
__device__ __forceinline__ bool dbit(const StepArgs &A, int32_t p)
{
    return (A.dbits[p >> 5] >> (p & 31)) & 1u;
}

// Round 1: one workgroup finishes whatever passes the grid left, then sets
// up the first check: the particles with a history (those of the listed
// candidates) become D.
__global__ __launch_bounds__(1024) void k_finish(StepArgs A)
{
    __shared__ PassShared S;
    __shared__ int s_t0;
    __shared__ int64_t s_c0;
    __shared__ int32_t s_pl;
    if (threadIdx.x == 0) {
        s_t0 = A.ctl[CTL_PASS];
        s_c0 = list_count(A, s_t0);
        s_pl = 0;
    }
    __syncthreads();
    const int t0 = s_t0;
    const int64_t c0 = s_c0;
    __syncthreads();
    wg_passes(A, t0, c0, S);
    int64_t mc = A.ctl[CTL_MEM];
    mc = mc < A.cap_acc ? mc : A.cap_acc;
    for (int64_t m = threadIdx.x; m < mc; m += blockDim.x) {
        const int32_t pp[2] = {A.M.i[m], A.M.j[m]};
        for (int u = 0; u < 2; ++u)
            if (atomicMin(&A.tmin[pp[u]], 0ull) == ~0ull) {
                A.plist[atomicAdd(&s_pl, 1)] = pp[u];
                set_dbit(A, pp[u]);
            }
    }
    wg_sync();
    if (threadIdx.x == 0) {
        A.ctl[CTL_NEWLO] = (int32_t)mc;
        A.ctl[CTL_PL] = s_pl;
        if (A.ctl[CTL_FREE] < 0) A.ctl[CTL_FREE] = 0;
    }
}

// ----------------------------------------------------------------------------
// Check of a round: every candidate touching a particle of D (whose history
// changed since the last check) is evaluated at its turn.
// ----------------------------------------------------------------------------

// The history of particle p at key (kp, ki): (tx, ty, tz) its velocity at that
// turn, rge the earliest record with key >= (kp, ki) (-1 if none), and
// (sx, sy, sz) its velocity at the step start.  Records go from the latest
// turn back, with decreasing keys (the guard only bounds a corrupted chain).
__device__ __forceinline__ void history_at(const StepArgs &A, int32_t p, uint64_t kp, uint64_t ki,
                                           double &tx, double &ty, double &tz, int32_t &rge,
                                           double &sx, double &sy, double &sz)
{
    tx = sx = A.vxs[p];
    ty = sy = A.vys[p];
    tz = sz = A.vzs[p];
    rge = -1;
    int32_t r = A.head[p];
    for (int64_t guard = 0; r >= 0 && guard < A.cap_rec; ++guard) {
        const uint64_t rp = A.R.prio[r], rq = A.R.idpair[r];
        const double ax = A.R.vx[r], ay = A.R.vy[r], az = A.R.vz[r];
        if (rp > kp || (rp == kp && rq >= ki)) { rge = r; tx = ax; ty = ay; tz = az; }
        sx = ax; sy = ay; sz = az;
        r = A.R.prev[r];
    }
}

// Candidate slot s of row a (target i, Morton order) at its turn, with the
// velocities the histories give there and at the step start.
struct TurnEval {
    double u, W, Pt, Ps;
    uint64_t kp, ki;
    int32_t j, ri;          // partner; earliest record of i at or after the key
};

template <bool PERIODIC, bool OVERLAP>
__device__ void eval_turn(const StepArgs &A, int32_t i, int32_t a, int32_t j, TurnEval &T)
{
    const uint32_t idi = A.ids[i], idj = A.ids[j];
    T.j = j;
    T.kp = direction_word(pair_draw(A.seed, A.step, idi, idj, PURPOSE_PRIORITY), idi < idj);
    T.ki = ((uint64_t)idi << 32) | idj;
    T.u = unit_from_word(direction_word(pair_draw(A.seed, A.step, idi, idj, PURPOSE_DECIDE),
                                        idi < idj));
    double tix, tiy, tiz, six, siy, siz, tjx, tjy, tjz, sjx, sjy, sjz;
    int32_t rj;
    history_at(A, i, T.kp, T.ki, tix, tiy, tiz, T.ri, six, siy, siz);
    history_at(A, j, T.kp, T.ki, tjx, tjy, tjz, rj, sjx, sjy, sjz);
    const double r = A.lphys * sqrt(sep2<PERIODIC>(A.xs[i], A.ys[i], A.zs[i], A.xs[j], A.ys[j],
                                                   A.zs[j], A.box));
    T.W = OVERLAP ? overlap_g(A.gtab, A.lphys * A.hsrt[i], A.lphys * A.hsrt[j], r)
                  : cubic_spline(r, A.lphys * A.h[a]);
    const bool allowed = pair_allowed(A, i, j);
    const double mj = mass_of(A, j), dta = A.dt[a];
    const double wt = A.vphys * rel_speed(tix, tiy, tiz, tjx, tjy, tjz);
    T.Pt = allowed ? pair_prob(mj, sigma_of(A, wt), wt, T.W, dta) : 0.0;
    const double ws = A.vphys * rel_speed(six, siy, siz, sjx, sjy, sjz);
    T.Ps = allowed ? pair_prob(mj, sigma_of(A, ws), ws, T.W, dta) : 0.0;
}

template <bool PERIODIC, bool OVERLAP>
__device__ void check_candidate(const StepArgs &A, int32_t i, int32_t a, int s, int32_t j)
{
    TurnEval T;
    eval_turn<PERIODIC, OVERLAP>(A, i, a, j, T);
    const int64_t ci = (int64_t)a * A.stride + s;
    const bool listed = T.ri >= 0 && A.R.prio[T.ri] == T.kp && A.R.idpair[T.ri] == T.ki;
    const bool kicked = listed && (A.R.info[T.ri] & 1u);
    const uint32_t depth = kicked ? A.R.info[T.ri] >> 8 : 0u;
    const bool flag_t = fabs(T.Pt - T.u) < A.band, flag_s = fabs(T.Ps - T.u) < A.band;
    if (!listed && T.u < T.Pt) {
        // accepts at its turn but did not take it: list it for the next round
        const int32_t pos = atomicAdd(&A.ctl[CTL_MEM], 1);
        if (pos < A.cap_acc) {
            A.M.i[pos] = i; A.M.j[pos] = T.j; A.M.cand[pos] = (int32_t)ci;
            A.M.u[pos] = T.u; A.M.W[pos] = T.W; A.M.dt[pos] = A.dt[a];
            A.M.prio[pos] = T.kp; A.M.idpair[pos] = T.ki; A.M.rec[pos] = -1;
        } else {
            atomicOr(A.derr, DERR_OVERFLOW);
        }
    }
    if (flag_t || flag_s) {
        // counted again at the end of the step with the final histories
        const int32_t f = atomicAdd(&A.ctl[CTL_FLAG], 1);
        if (f < SIDM_FLAG_CAP) { A.flist[2 * f] = i; A.flist[2 * f + 1] = (int32_t)ci; }
        else atomicOr(A.derr, DERR_OVERFLOW);
    }
    if (A.cand_info)
        A.cand_info[ci] = (T.u < T.Ps ? SIDM_CAND_ACCEPT0 : 0u) | (flag_t ? SIDM_CAND_FLAGGED : 0u) |
                          (kicked ? (SIDM_CAND_SCATTER | (depth << 8)) : 0u);
}

// The check's scan: every candidate whose target or partner is in D, each
// once; rows in Morton order (spatially close targets, so that the D bits of
// their partners share cache lines).  The whole workgroup calls it: each
// round of the loop scans blockDim candidates and queues the hits in LDS;
// whenever blockDim hits are queued they are evaluated with every thread
// busy (in the first round about one candidate in a hundred hits on the
// 256^3 box: evaluated where found, most lanes of a wavefront would wait).
constexpr int kScanU = 8;          // candidates a thread scans per round of the loop
static_assert(kScanU % 4 == 0, "the row-wise scan takes four candidates of a row a lane");

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_or_u32(unsigned int);

// Summaries of the row blocks a round of the row-wise scan covers (kBlock
// threads, kScanU / 4 rows a lane: kScanU / 4 blocks of SIDM_SUM_U).  Each
// wavefront lists the buckets outside a block's window that it saw, each
// once; the block's writer merges the wavefronts' lists.
constexpr int kSumPer = kScanU / 4;
constexpr int kSumWaves = kBlock / 64;
static_assert(kBlock * 4 == SIDM_SUM_U, "a row of the row-wise scan's lanes covers one block");
static_assert(kSumWaves * SIDM_SUM_OUT <= 64 && kSumPer <= kSumWaves, "a wavefront merges a block's lists");
struct SumLds {
    uint32_t m[kSumPer][2];
    int cnt[kSumPer][kSumWaves];                      // > SIDM_SUM_OUT: too many
    int32_t out[kSumPer][kSumWaves][SIDM_SUM_OUT];
};

__device__ __forceinline__ void sum_reset(SumLds *S, int tid)
{
    if (tid < kSumPer) { S->m[tid][0] = 0u; S->m[tid][1] = 0u; }
}

// The distinct values of the lanes' pending entries v[e] (bit e of pend), at
// most SIDM_SUM_OUT + 1 of them, one a round: lane r gets the r-th in found;
// returns their number.
template <int E>
__device__ __forceinline__ int wave_distinct(const int32_t (&v)[E], uint32_t pend, int32_t &found)
{
    const int lane = threadIdx.x & 63;
    int nf = 0;
    for (; nf <= SIDM_SUM_OUT; ++nf) {
        const uint64_t any = __ballot(pend != 0u);
        if (any == 0ull) break;
        int32_t mine = -1;
#pragma unroll
        for (int e = E - 1; e >= 0; --e)
            if ((pend >> e) & 1u) mine = v[e];
        const int32_t bk = __builtin_amdgcn_readlane(mine, __ffsll((long long)any) - 1);
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (((pend >> e) & 1u) && v[e] == bk) pend &= ~(1u << e);
        if (lane == nf) found = bk;
    }
    return nf;
}

// A lane's buckets v (-1: none) into block p's summary: those within 32 of
// base into the mask, the others into this wavefront's list.
__device__ __forceinline__ void sum_add(SumLds *S, int p, int32_t base, const int32_t (&v)[5])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t mlo = 0u, mhi = 0u, pend = 0u;
#pragma unroll
    for (int e = 0; e < 5; ++e) {
        if (v[e] < 0) continue;
        const int32_t rel = v[e] - base + 32;
        if (rel >= 0 && rel < 32) mlo |= 1u << rel;
        else if (rel >= 32 && rel < 64) mhi |= 1u << (rel - 32);
        else pend |= 1u << e;
    }
    mlo = __ockl_wfred_or_u32(mlo);
    mhi = __ockl_wfred_or_u32(mhi);
    if (lane == 0) {
        if (mlo) atomicOr(&S->m[p][0], mlo);
        if (mhi) atomicOr(&S->m[p][1], mhi);
    }
    int32_t found = -1;
    const int nf = wave_distinct<5>(v, pend, found);
    if (lane < nf && lane < SIDM_SUM_OUT) S->out[p][w][lane] = found;
    if (lane == 0) S->cnt[p][w] = nf;
}

// Wavefront p of the workgroup merges block p's lists and writes the
// summary of block blk.
__device__ __forceinline__ void sum_write(const StepArgs &A, const SumLds *S, int p, int64_t blk, int sh)
{
    const int lane = threadIdx.x & 63;
    const int w = lane / SIDM_SUM_OUT, r = lane % SIDM_SUM_OUT;
    bool over = false;
#pragma unroll
    for (int q = 0; q < kSumWaves; ++q) over = over || S->cnt[p][q] > SIDM_SUM_OUT;
    int32_t v[1] = {-1};
    if (w < kSumWaves && r < S->cnt[p][w]) v[0] = S->out[p][w][r];
    int32_t found = -1;
    const int nf = wave_distinct<1>(v, v[0] >= 0 ? 1u : 0u, found);
    over = over || nf > SIDM_SUM_OUT;
    int32_t *o = A.csum + blk * SIDM_SUM_WORDS;
    if (!over && lane < nf) o[4 + lane] = found;
    if (lane == 32) o[0] = (int32_t)S->m[p][0];
    if (lane == 33) o[1] = (int32_t)S->m[p][1];
    if (lane == 34) o[2] = A.tlist[(blk * SIDM_SUM_U) >> sh] >> SIDM_DBUCKET_SHIFT;
    if (lane == 35) o[3] = over ? -1 : nf;
}

template <bool PERIODIC, bool OVERLAP, bool BUILD = false>
__device__ void check_scan(const StepArgs &A, int64_t first_chunk, int64_t chunk_stride,
                           int32_t *q, int &qn, SumLds *S = nullptr)
{
    const int nth = blockDim.x, tid = threadIdx.x;
    const int64_t nt = *A.nt_dev;
    const int64_t total = nt * A.stride;
    auto evaluate = [&](int64_t c) {
        const int64_t b = c / A.stride;
        const int s = (int)(c - b * A.stride);
        const int32_t a = A.slot[b];
        const int32_t j = partner(A, c, (int64_t)a * A.stride + s);
        check_candidate<PERIODIC, OVERLAP>(A, A.tlist[b], a, s, j);
    };
    const int sh = stride_shift(A.stride);
    if (tid == 0) qn = 0;
    if (BUILD) sum_reset(S, tid);
    __syncthreads();
    // chunks of nth * kScanU candidates; a thread takes kScanU of a chunk,
    // nth apart, with their loads independent of each other
    for (int64_t c0 = first_chunk; c0 < total; c0 += chunk_stride) {
        int64_t cc[kScanU];
        bool hit[kScanU];
        if (!OVERLAP && A.jsort && sh >= 2) {
            // rows in the tree's order, k = 2^sh >= 4: a lane takes four
            // candidates of a row (k / 4 lanes a row, kScanU / 4 rows a lane),
            // the target tlist[b] and its D bit once, the partners jsort[c]
            const int lsh = sh - 2;
            const int L = 1 << lsh;
            const int64_t b0 = c0 >> sh;
            const int rows_pass = nth >> lsh;
            int32_t jv[kScanU];
            bool di[kScanU / 4];
#pragma unroll
            for (int p = 0; p < kScanU / 4; ++p) {
                const int64_t b = b0 + p * rows_pass + (tid >> lsh);
                const int l = tid & (L - 1);
                const bool ok = b < nt;
                const int32_t i = ok ? A.tlist[b] : 0;
                // four consecutive entries of the row, one 16-byte load
                const int64_t c4 = (b << sh) + 4 * l;
                const int4 q = ok ? *(const int4 *)(A.jsort + c4) : make_int4(-1, -1, -1, -1);
                jv[p * 4 + 0] = q.x; jv[p * 4 + 1] = q.y; jv[p * 4 + 2] = q.z; jv[p * 4 + 3] = q.w;
#pragma unroll
                for (int u = 0; u < 4; ++u) cc[p * 4 + u] = c4 + u;
                di[p] = ok && dbit(A, i);
            }
#pragma unroll
            for (int e = 0; e < kScanU; ++e) hit[e] = jv[e] >= 0 && (di[e / 4] || dbit(A, jv[e]));
            if constexpr (BUILD) {
                // the summaries of this chunk's blocks (rows of the block's
                // lanes: p, the first target's bucket its base)
#pragma unroll
                for (int p = 0; p < kSumPer; ++p) {
                    const int64_t bf = b0 + p * rows_pass;
                    const int64_t b = bf + (tid >> lsh);
                    const int32_t base = A.tlist[bf < nt ? bf : 0] >> SIDM_DBUCKET_SHIFT;
                    int32_t v[5];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = jv[p * 4 + u] >= 0 ? jv[p * 4 + u] >> SIDM_DBUCKET_SHIFT : -1;
                    v[4] = b < nt ? A.tlist[b] >> SIDM_DBUCKET_SHIFT : -1;
                    sum_add(S, p, base, v);
                }
            }
        } else {
            int32_t jj[kScanU], ii[kScanU];
#pragma unroll
            for (int u = 0; u < kScanU; ++u) {
                const int64_t c = c0 + u * nth + tid;
                cc[u] = c;
                jj[u] = -1;
                ii[u] = 0;
                if (c < total) {
                    const int64_t b = row_of_cand(c, sh, A.stride, total);
                    const int s = (int)(c - b * A.stride);
                    if (!OVERLAP && A.jsort) {
                        jj[u] = A.jsort[c];
                        ii[u] = A.tlist[b];
                    } else {
                        const int32_t a = A.slot[b];
                        if (!OVERLAP || s < A.cnt[a]) {
                            jj[u] = partner(A, c, (int64_t)a * A.stride + s);
                            ii[u] = A.tlist[b];
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kScanU; ++u) hit[u] = jj[u] >= 0 && (dbit(A, jj[u]) || dbit(A, ii[u]));
        }
#pragma unroll
        for (int u = 0; u < kScanU; ++u)
            if (hit[u]) q[atomicAdd(&qn, 1)] = (int32_t)cc[u];
        __syncthreads();
        if constexpr (BUILD) {
            const int p = tid >> 6;
            const int64_t blk = c0 / SIDM_SUM_U + p;
            if (p < kSumPer && blk * SIDM_SUM_U < total) sum_write(A, S, p, blk, sh);
        }
        int n_q = qn;
        while (n_q >= nth) {
            evaluate(q[n_q - nth + tid]);
            n_q -= nth;
        }
        __syncthreads();
        if (tid == 0) qn = n_q;
        if (BUILD) sum_reset(S, tid);
        __syncthreads();
    }
    const int n_q = qn;
    if (tid < n_q) evaluate(q[tid]);
    __syncthreads();
}

// Does the block whose summary is s hold a candidate touching D?  False only
// if none of its buckets holds a particle of D.
__device__ __forceinline__ bool block_meets_d(const StepArgs &A, const int32_t *s)
{
    const int4 h = *(const int4 *)s;
    const int nout = h.w;
    if (nout < 0) return true;
    const uint64_t mask = (uint64_t)(uint32_t)h.x | ((uint64_t)(uint32_t)h.y << 32);
    if (mask) {
        const int64_t b0 = (int64_t)h.z - 32;          // the bucket of mask bit 0
        const int64_t w0 = b0 >= 0 ? (b0 >> 5) : -((31 - b0) >> 5);
        const int o = (int)(b0 - w0 * 32);
        uint64_t wd[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int64_t w = w0 + e;
            wd[e] = (w >= 0 && w < A.nbw) ? A.bbits[w] : 0u;
        }
        const uint64_t lo = wd[0] | (wd[1] << 32);
        const uint64_t win = o == 0 ? lo : (lo >> o) | (wd[2] << (64 - o));
        if (win & mask) return true;
    }
    for (int e = 0; e < nout; ++e) {
        const int32_t bk = s[4 + e];
        if ((A.bbits[bk >> 5] >> (bk & 31)) & 1u) return true;
    }
    return false;
}

// The check's scan with block summaries (rows in the tree's order of a
// power of two entries, k <= SIDM_SUM_U): the blocks are tested against the
// bucket bits of D, nth at a time, and only the blocks that may hold a
// candidate touching D are scanned, nth / 256 at once, 256 threads of four
// candidates of a row each; hits queue and are evaluated as in check_scan.
template <bool PERIODIC>
__device__ void check_blocks(const StepArgs &A, int64_t g0, int64_t g_stride, int gsz, int32_t *q,
                             int &qn, int32_t *sb, int &sbn)
{
    const int nth = blockDim.x, tid = threadIdx.x;
    const int64_t nt = *A.nt_dev;
    const int64_t total = nt * A.stride;
    const int64_t nblocks = (total + SIDM_SUM_U - 1) / SIDM_SUM_U;
    const int sh = stride_shift(A.stride);
    const int lsh = sh - 2;
    const int L = 1 << lsh;
    const int G = nth >> 8;
    constexpr int PB = 2;
    static_assert(4 * PB <= kScanU, "a round queues at most kScanU hits a thread");
    auto evaluate = [&](int64_t c) {
        const int64_t b = c >> sh;
        const int s = (int)(c - (b << sh));
        const int32_t a = A.slot[b];
        const int32_t j = partner(A, c, (int64_t)a * A.stride + s);
        check_candidate<PERIODIC, false>(A, A.tlist[b], a, s, j);
    };
    if (tid == 0) qn = 0;
    __syncthreads();
    for (int64_t g = g0; g * gsz < nblocks; g += g_stride) {
        if (tid == 0) sbn = 0;
        __syncthreads();
        const int64_t u = g * gsz + tid;
        if (tid < gsz && u < nblocks && block_meets_d(A, A.csum + u * SIDM_SUM_WORDS)) sb[atomicAdd(&sbn, 1)] = (int32_t)u;
        __syncthreads();
        const int nb = sbn;
        // PB blocks a round for a workgroup of 256 threads (G * PB for more)
        for (int h0 = 0; h0 < nb; h0 += G * PB) {
            const int t = tid & 255;
            int64_t cc[4 * PB];
            bool hit[4 * PB];
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                const int h = h0 + p * G + (tid >> 8);
                int32_t jv[4];
                bool di = false;
#pragma unroll
                for (int e = 0; e < 4; ++e) { cc[p * 4 + e] = 0; jv[e] = -1; }
                if (h < nb) {
                    const int64_t b = (((int64_t)sb[h] * SIDM_SUM_U) >> sh) + (t >> lsh);
                    if (b < nt) {
                        const int l = t & (L - 1);
                        di = dbit(A, A.tlist[b]);
                        const int64_t c4 = (b << sh) + 4 * l;
                        const int4 q = *(const int4 *)(A.jsort + c4);
                        jv[0] = q.x; jv[1] = q.y; jv[2] = q.z; jv[3] = q.w;
#pragma unroll
                        for (int e = 0; e < 4; ++e) cc[p * 4 + e] = c4 + e;
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) hit[p * 4 + e] = jv[e] >= 0 && (di || dbit(A, jv[e]));
            }
#pragma unroll
            for (int e = 0; e < 4 * PB; ++e)
                if (hit[e]) q[atomicAdd(&qn, 1)] = (int32_t)cc[e];
            __syncthreads();
            int n_q = qn;
            while (n_q >= nth) {
                evaluate(q[n_q - nth + tid]);
                n_q -= nth;
            }
            __syncthreads();
            if (tid == 0) qn = n_q;
            __syncthreads();
        }
    }
    const int n_q = qn;
    if (tid < n_q) evaluate(q[tid]);
    __syncthreads();
}

// blocks a workgroup of the grid check tests at once: few, so that the
// groups of a large step outnumber the workgroups and spread over every XCD
// (consecutive workgroups go to different XCDs), and the blocks that meet D,
// which cluster, spread over many workgroups (64, 32, 16, 8 measured: 16)
constexpr int kCheckGroup = 16;

// The block summaries are tested only while few buckets hold a particle of
// D (at most a quarter of them): with more, most blocks would be scanned
// anyway and the plain scan is faster.
__device__ __forceinline__ bool use_blocks(const StepArgs &A, int32_t dbk)
{
    return A.csum && (int64_t)dbk * 4 <= A.nbw * 32;
}

// The index buckets holding a particle of D, from its bits: one thread per
// bucket (SIDM_DBUCKET particles, 2^SIDM_DBUCKET_SHIFT / 32 words of bits),
// a bucket word per half wavefront; the count of such buckets into CTL_DBK
// (zeroed by the round that set D).
__device__ __forceinline__ int dbucket_word(const StepArgs &A, int64_t bk)
{
    constexpr int W = (1 << SIDM_DBUCKET_SHIFT) / 32;
    const int64_t ndw = (A.n + 31) / 32;
    const int64_t w0 = bk * W;
    uint32_t any = 0u;
    if (w0 + W <= ndw) {
#pragma unroll
        for (int e = 0; e < W; e += 4) {
            const uint4 d = *(const uint4 *)(A.dbits + w0 + e);
            any |= d.x | d.y | d.z | d.w;
        }
    } else {
        for (int64_t w = w0; w < ndw; ++w) any |= A.dbits[w];
    }
    return any != 0u;
}

__global__ __launch_bounds__(kBlock) void k_dbuckets(StepArgs A)
{
    if (load_i32(&A.ctl[CTL_DONE])) return;
    const int lane = threadIdx.x & 63;
    const int64_t nb = A.nbw * 32;
    for (int64_t b0 = xcd_stride_block() * (int64_t)kBlock + (threadIdx.x & ~63); b0 < nb;
         b0 += (int64_t)gridDim.x * kBlock) {
        const int64_t bk = b0 + lane;
        const uint64_t m = __ballot(bk < nb && dbucket_word(A, bk));
        if (lane == 0) {
            A.bbits[b0 >> 5] = (uint32_t)m;
            if (m) atomicAdd(&A.ctl[CTL_DBK], __popcll(m));
        } else if (lane == 32 && (b0 >> 5) + 1 < A.nbw) {
            A.bbits[(b0 >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
}

// The first check (BUILD) scans every candidate and writes the block
// summaries on the way; later checks scan the blocks that may hold a
// candidate touching D while few buckets do.
template <bool PERIODIC, bool OVERLAP, bool BUILD>
__global__ __launch_bounds__(kBlock) void k_check(StepArgs A)
{
    __shared__ int32_t q[(kScanU + 1) * kBlock];
    __shared__ int32_t sb[kBlock];
    __shared__ int qn, sbn;
    __shared__ SumLds S;
    if (A.ctl[CTL_DONE]) return;
    if constexpr (BUILD && !OVERLAP) {
        check_scan<PERIODIC, false, true>(A, xcd_stride_block() * (int64_t)kBlock * kScanU,
                                          (int64_t)gridDim.x * kBlock * kScanU, q, qn, &S);
    } else {
        if (!OVERLAP && use_blocks(A, A.ctl[CTL_DBK]))
            check_blocks<PERIODIC>(A, blockIdx.x, gridDim.x, kCheckGroup, q, qn, sb, sbn);
        else
            check_scan<PERIODIC, OVERLAP>(A, xcd_stride_block() * (int64_t)kBlock * kScanU,
                                          (int64_t)gridDim.x * kBlock * kScanU, q, qn);
    }
}

// ----------------------------------------------------------------------------
// Re-round: list the newly accepting candidates, rewind the turns they can
// affect and take them again.  One workgroup.  The rewound particles become
// the next check's D.
// ----------------------------------------------------------------------------
struct RoundShared {
    PassShared ps;
    int go;
    int32_t lo, hi;          // newly listed candidates [lo, hi)
    int32_t dl;              // candidates to replay (in work list 0)
    int32_t pl;              // particles to rewind (in plist)
    int32_t f0, f1;          // frontier of the closure
};

__device__ void reround_body(const StepArgs &A, RoundShared &S)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    if (tid == 0) {
        S.go = 0;
        if (!load_i32(&A.ctl[CTL_DONE])) {
            const int32_t mc = load_i32(&A.ctl[CTL_MEM]);
            const int32_t lo = load_i32(&A.ctl[CTL_NEWLO]);
            const unsigned int bad = __hip_atomic_load(A.derr, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) &
                                     (DERR_OVERFLOW | DERR_HISTORY | DERR_STALL);
            if (mc > A.cap_acc || mc <= lo || bad) {
                // nothing newly listed: the last check saw the serial order
                // (or a buffer overflowed, which is latched: stop)
                A.ctl[CTL_DONE] = 1;
            } else {
                S.go = 1; S.lo = lo; S.hi = mc;
            }
        }
    }
    __syncthreads();
    if (!S.go) return;
    // the last check's D is done with
    const int32_t old_pl = load_i32(&A.ctl[CTL_PL]);
    for (int32_t q = tid; q < old_pl; q += nth) {
        const int32_t p = A.plist[q];
        atomicExch(&A.tmin[p], ~0ull);
        clear_dbit(A, p);
    }
    // seeds: the newly listed candidates
    const int32_t n0 = S.hi - S.lo;
    for (int32_t q = tid; q < n0; q += nth) {
        A.mmark[S.lo + q] = 1;
        A.wl0[q] = S.lo + q;
    }
    if (tid == 0) { S.dl = n0; S.pl = 0; S.f0 = 0; S.f1 = n0; }
    wg_sync();
    // closure: a turn later than a replayed turn of one of its particles is
    // replayed too.  tmin[p] is the smallest priority replayed at p; every
    // turn of p with a priority at least that is marked (equal priorities
    // with a smaller ID pair included, which only replays one turn more).
    while (true) {
        for (int32_t q = S.f0 + tid; q < S.f1; q += nth) {
            const int32_t m = A.wl0[q];
            const unsigned long long pr = A.M.prio[m];
            const int32_t pp[2] = {A.M.i[m], A.M.j[m]};
            for (int u = 0; u < 2; ++u) {
                const unsigned long long old = atomicMin(&A.tmin[pp[u]], pr);
                if (old == ~0ull) {
                    A.plist[atomicAdd(&S.pl, 1)] = pp[u];
                    set_dbit(A, pp[u]);
                }
            }
        }
        wg_sync();
        for (int32_t q = tid; q < S.pl; q += nth) {
            const int32_t p = A.plist[q];
            const unsigned long long tp = load_u64(&A.tmin[p]);
            int32_t r = A.head[p];
            for (int64_t guard = 0; r >= 0 && guard < A.cap_rec && A.R.prio[r] >= tp; ++guard) {
                const int32_t m2 = A.R.mem[r];
                if (atomicCAS(&A.mmark[m2], 0, 1) == 0) A.wl0[atomicAdd(&S.dl, 1)] = m2;
                r = A.R.prev[r];
            }
        }
        wg_sync();
        const bool grew = S.dl > S.f1;
        __syncthreads();
        if (!grew) break;
        if (tid == 0) { S.f0 = S.f1; S.f1 = S.dl; }
        __syncthreads();
    }
    // rewind: each particle back to its velocity (and state) before the
    // earliest marked turn, its history cut there; tmin stays set, marking
    // the particle as one of the next check's D
    for (int32_t q = tid; q < S.pl; q += nth) {
        const int32_t p = A.plist[q];
        const unsigned long long tp = load_u64(&A.tmin[p]);
        int32_t r = A.head[p], rr = -1;
        for (int64_t guard = 0; r >= 0 && guard < A.cap_rec && A.R.prio[r] >= tp; ++guard) {
            // a turn's records are cut together (its two particles both
            // rewind past it): the pair is freed once, at its first record
            if ((r & 1) == 0) A.rfree[atomicAdd(&A.ctl[CTL_FREE], 1)] = r >> 1;
            rr = r;
            r = A.R.prev[r];
        }
        A.head[p] = r;
        if (rr >= 0) {
            const double nx = A.R.vx[rr], ny = A.R.vy[rr], nz = A.R.vz[rr];
            A.vxs[p] = nx; A.vys[p] = ny; A.vzs[p] = nz;
            const int32_t op = A.perm[p];
            A.vx[op] = nx; A.vy[op] = ny; A.vz[op] = nz;
            if (A.model == SIDM_MODEL_TWO_STATE) {
                const uint8_t st = (uint8_t)((A.R.info[rr] >> 1) & 0x7fu);
                A.sts[p] = st;
                if (A.state) A.state[op] = st;
            }
        }
    }
    wg_sync();
    for (int32_t q = tid; q < S.dl; q += nth) {
        const int32_t m = A.wl0[q];
        atomicExch(&A.mmark[m], 0);
        const int32_t i = A.M.i[m], j = A.M.j[m];
        A.c1a[i] = ~0ull; A.c1a[j] = ~0ull;
        A.c2a[i] = ~0ull; A.c2a[j] = ~0ull;
    }
    wg_sync();
    wg_passes(A, 0, S.dl, S.ps);
    wg_sync();
    if (tid == 0) {
        A.ctl[CTL_NEWLO] = S.hi;
        A.ctl[CTL_PL] = S.pl;
        A.ctl[CTL_DBK] = 0;
        A.ctl[CTL_ROUNDS] += 1;
        // pops that found the free stack empty left the count below zero
        if (A.ctl[CTL_FREE] < 0) A.ctl[CTL_FREE] = 0;
    }
    wg_sync();
}

__global__ __launch_bounds__(1024) void k_reround(StepArgs A)
{
    __shared__ RoundShared S;
    reround_body(A, S);
}

// Rounds left after the grid launches: checks and re-rounds in one
// workgroup until no candidate is newly listed.  Every round lists at least
// one more candidate or ends, and the list is bounded, so the loop ends.
constexpr int kTailRounds = 1 << 16;       // far above any round count seen

template <bool PERIODIC, bool OVERLAP>
__global__ __launch_bounds__(1024) void k_tail(StepArgs A)
{
    __shared__ RoundShared S;
    __shared__ int s_done;
    __shared__ int32_t tq[(kScanU + 1) * 1024];
    __shared__ int32_t tsb[1024];
    __shared__ int tqn, tsbn;
    for (int round = 0;; ++round) {
        if (threadIdx.x == 0) {
            s_done = load_i32(&A.ctl[CTL_DONE]);
            if (!s_done && round >= kTailRounds) {
                atomicOr(A.derr, DERR_STALL);
                s_done = 1;
            }
        }
        __syncthreads();
        if (s_done) break;
        if (!OVERLAP && A.csum) {
            // the bucket bits of this round's D
            if (threadIdx.x == 0) tsbn = 0;
            __syncthreads();
            const int lane = threadIdx.x & 63;
            const int64_t nb = A.nbw * 32;
            for (int64_t b0 = threadIdx.x & ~63; b0 < nb; b0 += blockDim.x) {
                const uint64_t m = __ballot(b0 + lane < nb && dbucket_word(A, b0 + lane));
                if (lane == 0) {
                    A.bbits[b0 >> 5] = (uint32_t)m;
                    if (m) atomicAdd(&tsbn, __popcll(m));
                } else if (lane == 32 && (b0 >> 5) + 1 < A.nbw) {
                    A.bbits[(b0 >> 5) + 1] = (uint32_t)(m >> 32);
                }
            }
            __syncthreads();
            const int dbk = tsbn;
            __syncthreads();
            if (use_blocks(A, dbk)) check_blocks<PERIODIC>(A, 0, 1, 1024, tq, tqn, tsb, tsbn);
            else check_scan<PERIODIC, OVERLAP>(A, 0, (int64_t)blockDim.x * kScanU, tq, tqn);
        } else {
            check_scan<PERIODIC, OVERLAP>(A, 0, (int64_t)blockDim.x * kScanU, tq, tqn);
        }
        wg_sync();
        reround_body(A, S);
        wg_sync();
    }
}

// End of the step, one workgroup: the kicks and the largest kick depth from
// the listed candidates' turns, and the flagged count corrected by the
// candidates a check saw flagged (at the step start or at their turn),
// evaluated again with the final histories (each once).
template <bool PERIODIC, bool OVERLAP>
__global__ __launch_bounds__(1024) void k_final_stats(StepArgs A)
{
    __shared__ unsigned long long s_ev;
    __shared__ long long s_df;
    __shared__ unsigned int s_dp;
    if (threadIdx.x == 0) { s_ev = 0; s_df = 0; s_dp = 0; }
    __syncthreads();
    int64_t mc = A.ctl[CTL_MEM];
    mc = mc < A.cap_acc ? mc : A.cap_acc;
    unsigned long long ev = 0;
    unsigned int dp = 0;
    for (int64_t m = threadIdx.x; m < mc; m += blockDim.x) {
        const int32_t r = A.M.rec[m];
        if (r < 0) continue;
        const uint32_t info = A.R.info[r];
        if (info & 1u) {
            ++ev;
            dp = (info >> 8) > dp ? (info >> 8) : dp;
        }
    }
    int nf = A.ctl[CTL_FLAG];
    nf = nf < SIDM_FLAG_CAP ? nf : SIDM_FLAG_CAP;
    long long df = 0;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
        const int32_t i = A.flist[2 * f], ci = A.flist[2 * f + 1];
        bool first = true;
        for (int g = 0; g < f && first; ++g) first = A.flist[2 * g + 1] != ci;
        if (!first) continue;
        const int32_t a = (int32_t)(ci / A.stride);
        const int32_t jc = A.ngb[ci];
        if (jc < 0 || jc >= A.n) continue;
        TurnEval T;
        eval_turn<PERIODIC, OVERLAP>(A, i, a, A.inv[jc], T);
        df += (long long)(fabs(T.Pt - T.u) < A.band) - (long long)(fabs(T.Ps - T.u) < A.band);
    }
    if (ev) atomicAdd(&s_ev, ev);
    if (df) atomicAdd((unsigned long long *)&s_df, (unsigned long long)df);
    if (dp) atomicMax(&s_dp, dp);
    __syncthreads();
    if (threadIdx.x == 0) {
        A.st->n_events = s_ev;
        A.st->n_flagged += (unsigned long long)s_df;
        A.st->n_passes = s_dp;
        A.st->n_rounds = 1u + (unsigned)A.ctl[CTL_ROUNDS];
    }
}

// Clears every history and the last check's D for the next step.
__global__ __launch_bounds__(kBlock) void k_step_final(StepArgs A)
{
    int64_t nr = A.ctl[CTL_REC];
    nr = nr < A.cap_rec ? nr : A.cap_rec;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nr;
         r += (int64_t)gridDim.x * blockDim.x)
        A.head[A.R.part[r]] = -1;
    const int32_t np = A.ctl[CTL_PL];
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < np;
         q += (int64_t)gridDim.x * blockDim.x) {
        A.tmin[A.plist[q]] = ~0ull;
        clear_dbit(A, A.plist[q]);
    }
}

// Zeroes the step's statistics and control words; with nt_dev given, the
// candidate count is the number of targets times k.
__global__ void k_step_reset(DevStats *st, int32_t *ctl, const int32_t *nt_dev, int k)
{
    if (threadIdx.x == 0) {
        DevStats z = {};
        if (nt_dev) z.n_cand = (unsigned long long)(*nt_dev) * (unsigned long long)k;
        *st = z;
        for (int q = 0; q < 16; ++q) ctl[q] = 0;
    }
}

// ----------------------------------------------------------------------------
// Per-pair timestep (Eq. sidm_timestep) with the current velocities.  One
// thread per (target, neighbour) and a shuffle max over the target's lanes
// when n_ngb is a power of two up to 64; one thread per target otherwise.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double pair_rate(const StepArgs &A, double vix, double viy, double viz,
                                            int32_t j)
{
    if (j < 0) { atomicOr(A.derr, DERR_INDEX); return 0.0; }
    const double w = A.vphys * rel_speed(vix, viy, viz, A.vxs[j], A.vys[j], A.vzs[j]);
    return w * sigma_of(A, w);
}

__device__ __forceinline__ double dt_from_rate(const StepArgs &A, int32_t i, double h, double rmax,
                                               double c_sidm)
{
    const double W0 = cubic_spline(0.0, A.lphys * h);
    return rmax > 0.0 ? (2.0 * c_sidm) / ((mass_of(A, i) * W0) * rmax) : INFINITY;
}

// The velocities as (vx, vy, vz, 0) records of 32 bytes (in the phase
// buffer, which the timestep does not otherwise use), for the timestep's
// gathers of partners: two 16-byte loads of one line instead of three
// gathers of three lines.
__global__ __launch_bounds__(kBlock) void k_vel_aos(int64_t n, const double *vx, const double *vy,
                                                   const double *vz, double2 *out)
{
    // a lane a half record: (vx, vy) or (vz, 0)
    for (int64_t t = xcd_stride_block() * (int64_t)kBlock + threadIdx.x; t < 2 * n;
         t += (int64_t)gridDim.x * kBlock) {
        const int64_t q = t >> 1;
        out[t] = (t & 1) ? make_double2(vz[q], 0.0) : make_double2(vx[q], vy[q]);
    }
}

// A row of k (a power of two, at most 64) candidates per k / U lanes, U =
// min(4, k) candidates a lane (lane l takes l, l + k/U, ...); the row's
// maximum in registers, then by shuffles.  CONST: sigma is constant, so
// w sigma rises with w^2 and, sqrt and the products rounding monotonically,
// the largest rate is that of the largest w^2: the lanes carry w^2 and the
// row's first lane takes one square root (the same value as the largest of
// the rates).  CONST reads the partners' velocities from those records.
template <bool CONST, bool REC>
__global__ __launch_bounds__(kBlock) void k_timestep_group(StepArgs A, double c_sidm, double *dt_out)
{
    constexpr int UMAX = 4;
    const int64_t nt = *A.nt_dev;
    const int k = A.k;
    const int U = k < UMAX ? k : UMAX;
    const int L = k / U;                      // lanes per row (a power of two)
    const int lsh = __ffs(L) - 1;
    const int64_t total = nt << lsh;          // lanes in all
    for (int64_t t0 = xcd_stride_block() * (int64_t)blockDim.x; t0 < total;
         t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        const bool in = t < total;
        const int64_t b = in ? t >> lsh : 0;
        const int l = (int)(t & (L - 1));
        double v = CONST ? -1.0 : 0.0;
        int32_t i = 0, a = 0;
        if (in) {
            i = A.tlist[b];
            a = A.slot[b];
            const double vix = A.vxs[i], viy = A.vys[i], viz = A.vzs[i];
            int32_t jj[UMAX];
#pragma unroll
            for (int u = 0; u < UMAX; ++u) {
                const int s = l + u * L;
                jj[u] = u < U ? partner(A, b * k + s, (int64_t)a * k + s) : -2;
            }
#pragma unroll
            for (int u = 0; u < UMAX; ++u) {
                const int32_t j = jj[u];
                if (j == -2) continue;
                if constexpr (CONST) {
                    if (j < 0) {
                        atomicOr(A.derr, DERR_INDEX);
                    } else {
                        double vjx, vjy, vjz;
                        if constexpr (REC) {
                            const double4 vj = A.vaos[j];
                            vjx = vj.x; vjy = vj.y; vjz = vj.z;
                        } else {
                            vjx = A.vxs[j]; vjy = A.vys[j]; vjz = A.vzs[j];
                        }
                        const double dx = vix - vjx, dy = viy - vjy, dz = viz - vjz;
                        const double w2 = (dx * dx + dy * dy) + dz * dz;
                        v = w2 > v ? w2 : v;
                    }
                } else {
                    const double r = pair_rate(A, vix, viy, viz, j);
                    v = r > v ? r : v;
                }
            }
        }
        for (int off = 1; off < L; off <<= 1) {
            const double o = __shfl_xor(v, off);
            v = o > v ? o : v;
        }
        if (in && l == 0) {
            double rate = v;
            if constexpr (CONST) {
                rate = 0.0;
                if (v >= 0.0) {
                    const double w = A.vphys * sqrt(v);
                    rate = w * sigma_of(A, w);
                }
            }
            dt_out[a] = dt_from_rate(A, i, A.h[a], rate, c_sidm);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_timestep(StepArgs A, double c_sidm, double *dt_out)
{
    const int64_t nt = *A.nt_dev;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nt;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = A.tlist[b], a = A.slot[b];
        const double vix = A.vxs[i], viy = A.vys[i], viz = A.vzs[i];
        double rmax = 0.0;
        for (int s = 0; s < A.k; ++s) {
            const double r = pair_rate(A, vix, viy, viz,
                                       partner(A, b * A.k + s, (int64_t)a * A.k + s));
            rmax = r > rmax ? r : rmax;
        }
        dt_out[a] = dt_from_rate(A, i, A.h[a], rmax, c_sidm);
    }
}

// Overlap estimator: dt_i = 2 C_SIDM / (m_i max_j [g_ij(0) (w_ij sigma(w_ij)/m)])
// over the partners of the target's row.  A team of kTeamT lanes per target
// strides over its row; the maximum is taken by shuffles within the team.
constexpr int kTeamT = 32;

__global__ __launch_bounds__(kBlock) void k_timestep_overlap(StepArgs A, double c_sidm, double *dt_out)
{
    const int64_t nt = *A.nt_dev;
    const int tl = threadIdx.x % kTeamT;
    const int64_t teams = (int64_t)gridDim.x * (kBlock / kTeamT);
    for (int64_t b0 = (int64_t)blockIdx.x * (kBlock / kTeamT); b0 < nt; b0 += teams) {
        const int64_t b = b0 + threadIdx.x / kTeamT;     // team-uniform
        double qmax = 0.0;
        int32_t i = 0, a = 0;
        if (b < nt) {
            i = A.tlist[b];
            a = A.slot[b];
            const double vix = A.vxs[i], viy = A.vys[i], viz = A.vzs[i];
            const double hi = A.lphys * A.hsrt[i];
            const int len = A.cnt[a] < A.stride ? A.cnt[a] : A.stride;
            for (int s = tl; s < len; s += kTeamT) {
                const int32_t jc = A.ngb[(int64_t)a * A.stride + s];
                if (jc < 0 || jc >= A.n) { atomicOr(A.derr, DERR_INDEX); continue; }
                const int32_t j = A.inv[jc];
                const double w = A.vphys * rel_speed(vix, viy, viz, A.vxs[j], A.vys[j], A.vzs[j]);
                const double q = overlap_g0(A.gtab, hi, A.lphys * A.hsrt[j]) * (w * sigma_of(A, w));
                qmax = q > qmax ? q : qmax;
            }
        }
        for (int off = 1; off < kTeamT; off <<= 1) {
            const double o = __shfl_xor(qmax, off);
            qmax = o > qmax ? o : qmax;
        }
        if (b < nt && tl == 0)
            dt_out[a] = qmax > 0.0 ? (2.0 * c_sidm) / (mass_of(A, i) * qmax) : INFINITY;
    }
}

StepArgs make_args(sidm_ctx *c, sidm_particles *p, const int32_t *ngb, const double *h,
                   const double *dt, uint64_t seed, uint32_t step, uint32_t *cand_info)
{
    StepArgs A;
    A.xs = c->xs; A.ys = c->ys; A.zs = c->zs; A.ms = c->ms;
    A.vxs = c->vxs; A.vys = c->vys; A.vzs = c->vzs;
    A.ids = c->ids; A.sts = c->sts; A.perm = c->perm; A.inv = c->inv;
    A.vx = p ? p->vx : nullptr; A.vy = p ? p->vy : nullptr; A.vz = p ? p->vz : nullptr;
    A.state = p ? p->state : nullptr;
    A.tlist = c->tlist; A.slot = c->slot; A.nt_dev = c->nt_dev;
    A.ngb = ngb; A.h = h; A.dt = dt; A.cand_info = cand_info;
    A.M = c->mem;
    A.wl0 = c->wl[0]; A.wl1 = c->wl[1]; A.mmark = c->mmark; A.plist = c->plist; A.head = c->head;
    A.R = c->trec; A.tmin = c->tmin; A.cap_rec = c->cap_rec;
    A.rfree = c->rfree; A.dbits = c->dbits; A.flist = c->flist; A.jsort = nullptr;
    A.bbits = c->bbits; A.nbw = bucket_words(c->n); A.csum = nullptr; A.vaos = nullptr;
    A.erec = nullptr; A.recs = 0; A.verify_rows = 0;
    A.ctl = c->acc_count;
    A.c1a = c->claim1[0]; A.c1b = c->claim1[1]; A.c2a = c->claim2[0]; A.c2b = c->claim2[1];
    A.st = c->dstats; A.derr = c->derr;
    A.n = c->n; A.cap_acc = c->cap_acc;
    A.m_scalar = c->m_scalar;
    A.box = c->cfg.box; A.s0 = c->cfg.sigma0; A.w0 = c->cfg.w0;
    A.eps = c->cfg.eps; A.delta = c->cfg.delta; A.band = c->cfg.flag_band;
    A.seed = seed; A.step = step;
    A.k = c->cfg.n_ngb; A.periodic = c->cfg.periodic; A.xsec = c->cfg.xsec;
    A.model = c->cfg.model; A.has_mass = c->has_mass;
    A.xo = c->xo; A.yo = c->yo; A.zo = c->zo; A.nodes = c->nodes; A.band_p = c->cfg.band_p;
    A.xt_w = c->xt_w; A.xt_s = c->xt_s; A.xt_lw = c->xt_lw; A.xt_n = c->cfg.xsec_n;
    A.stride = A.k; A.cnt = nullptr; A.hsrt = c->hs; A.gtab = c->gtab;
    A.lphys = c->cfg.len_to_phys; A.vphys = c->cfg.vel_to_phys;
    return A;
}

// workgroups for n items, at most cap, a multiple of 8 (see xcd_stride_block)
int grid_for(int64_t n, int cap = 8192)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return grid8(g > cap ? cap : g);
}

// The step's rows in the tree's order: jsort[b * k + s] = sorted index of
// ngb[slot[b] * k + s] (-1, latched, for an index out of range).  When
// jsort holds the neighbour search's rows for this mapping (have = 1) an
// entry is only checked, perm[jsort] == ngb (partners of nearby targets lie
// close in the tree's order, so the gather stays in cache), and translated
// through inv where it differs; else every entry is translated.
__global__ __launch_bounds__(kBlock) void k_rows(StepArgs A, int have)
{
    const int64_t total = (int64_t)(*A.nt_dev) * A.stride;
    const int sh = stride_shift(A.stride);
    for (int64_t c = xcd_stride_block() * (int64_t)kBlock + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * kBlock) {
        const int64_t b = row_of_cand(c, sh, A.stride, total);
        const int s = (int)(c - b * A.stride);
        const int32_t jc = A.ngb[(int64_t)A.slot[b] * A.stride + s];
        int32_t j = have ? A.jsort[c] : -1;
        if (j >= 0 && j < A.n && A.perm[j] == jc) continue;
        j = -1;
        if (jc >= 0 && jc < A.n) j = A.inv[jc];
        else atomicOr(A.derr, DERR_INDEX);
        A.jsort[c] = j;
    }
}

// k_rows with four consecutive entries of a row per lane and 16-byte loads
// and stores (rows of a multiple of 4 entries, ngb 16-byte aligned).
__global__ __launch_bounds__(kBlock) void k_rows4(StepArgs A, int have)
{
    const int64_t total = (int64_t)(*A.nt_dev) * A.stride;
    const int64_t nq = total >> 2;
    const int sh = stride_shift(A.stride);
    for (int64_t q = xcd_stride_block() * (int64_t)kBlock + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * kBlock) {
        const int64_t c = q << 2;
        const int64_t b = row_of_cand(c, sh, A.stride, total);
        const int s = (int)(c - b * A.stride);
        const int4 g = *(const int4 *)(A.ngb + (int64_t)A.slot[b] * A.stride + s);
        const int4 h = have ? *(const int4 *)(A.jsort + c) : make_int4(-1, -1, -1, -1);
        const int32_t jc[4] = {g.x, g.y, g.z, g.w};
        int32_t j[4] = {h.x, h.y, h.z, h.w};
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = j[u] >= 0 && j[u] < A.n;
            ok[u] = in && A.perm[in ? j[u] : 0] == jc[u];
        }
        if (ok[0] && ok[1] && ok[2] && ok[3]) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ok[u]) continue;
            j[u] = -1;
            if (jc[u] >= 0 && jc[u] < A.n) j[u] = A.inv[jc[u]];
            else atomicOr(A.derr, DERR_INDEX);
        }
        *(int4 *)(A.jsort + c) = make_int4(j[0], j[1], j[2], j[3]);
    }
}

template <bool P, bool M, bool O = false>
void run_scatter(sidm_ctx *c, const StepArgs &A, int64_t n_active, hipStream_t s)
{
    const int64_t total = n_active * A.stride;
    k_step_reset<<<1, 64, 0, s>>>(A.st, A.ctl, O ? nullptr : A.nt_dev, A.k);
    phase_begin(c, PH_EVAL);
    // at least as many workgroups as are resident at once (the staging
    // buffer's LDS allows six per CU), more for long candidate lists (about
    // 2048 candidates a workgroup, at most 8192 workgroups: more cost more
    // in flushes and statistics atomics than they gain), each striding over
    // the candidates
    int64_t ge = total / 2048;
    ge = ge > 8192 ? 8192 : ge;
    const int geval = ge > kEvalGrid ? grid8(ge) : grid_for(total, kEvalGrid);
    if (!M && !O && A.jsort && A.stride >= 4 && (A.stride & (A.stride - 1)) == 0) {
        // rows of four candidates a lane: a quarter of the threads
        int64_t gr = total / 4 / 2048;
        gr = gr > 8192 ? 8192 : gr;
        const int gevr = gr > kEvalGrid ? grid8(gr) : grid_for(total / 4, kEvalGrid);
        // partner records when the gathers they save outweigh writing one
        // for every particle (at least 8 candidates a particle) and the
        // launch (2^20 candidates)
        if (A.recs) {
            StepArgs E = A;
            E.erec = (const double2 *)c->phase;
            k_eval_recs<<<grid_for(4 * A.n, 8192), kBlock, 0, s>>>(A, (double2 *)c->phase);
            if (A.verify_rows) k_eval_rows<P, true, true><<<gevr, kBlock, 0, s>>>(E);
            else k_eval_rows<P, true, false><<<gevr, kBlock, 0, s>>>(E);
        } else {
            k_eval_rows<P, false, false><<<gevr, kBlock, 0, s>>>(A);
        }
    } else {
        if (A.verify_rows)       // not reached (the rows form is taken whenever records are)
            k_rows<<<grid_for(total, 8192), kBlock, 0, s>>>(A, 1);
        k_eval<P, M, O><<<geval, kBlock, 0, s>>>(A);
    }
    phase_end(c, PH_EVAL);
    const int g = grid_for(A.cap_acc < total ? A.cap_acc : total, 2048);
    phase_begin(c, PH_RESOLVE);
    // round 1: the turns of the candidates accepted at the step start
    for (int t = 0; t < kMultiPasses; ++t) {
        k_claim1<<<g, kBlock, 0, s>>>(A, t);
        k_claim2<<<g, kBlock, 0, s>>>(A, t);
        k_resolve<<<g, kBlock, 0, s>>>(A, t);
    }
    k_finish<<<1, 1024, 0, s>>>(A);
    // checks and re-rounds until no candidate is newly listed (the kernels of
    // rounds after that return at once)
    int64_t dmax = 2 * (A.cap_acc < total ? A.cap_acc : total);
    dmax = dmax < A.n ? dmax : A.n;
    const int gcheck = grid_for((total + kScanU - 1) / kScanU, 8192);
    for (int r = 0; r < c->dev_rounds; ++r) {
        if (r == 0 && A.csum) {
            k_check<P, O, true><<<gcheck, kBlock, 0, s>>>(A);
        } else {
            if (A.csum) k_dbuckets<<<grid_for(A.nbw * 32, 1024), kBlock, 0, s>>>(A);
            k_check<P, O, false><<<gcheck, kBlock, 0, s>>>(A);
        }
        k_reround<<<1, 1024, 0, s>>>(A);
    }
    k_tail<P, O><<<1, 1024, 0, s>>>(A);
    k_final_stats<P, O><<<1, 1024, 0, s>>>(A);
    const int64_t nrec = A.cap_rec < 2 * total ? A.cap_rec : 2 * total;
    k_step_final<<<grid_for(nrec > dmax ? nrec : dmax, 1024), kBlock, 0, s>>>(A);
    phase_end(c, PH_RESOLVE);
}

}  // namespace

hipError_t launch_scatter(sidm_ctx *c, sidm_particles *p, int64_t n_active, const int32_t *ngb,
                          const double *h, const double *dt, uint64_t seed, uint32_t step,
                          uint32_t *cand_info)
{
    StepArgs A = make_args(c, p, ngb, h, dt, seed, step, cand_info);
    A.jsort = c->jsort;
    const int have = c->jsort_knn || c->jsort_ngb == ngb;
    const bool mixed = c->cfg.precision == SIDM_MIXED;
    const int st = A.stride;
    const int64_t cands = n_active * st;
    // the row-wise evaluation (rows of a power of two entries) gathers from
    // partner records when they outweigh writing one for every particle (at
    // least 8 candidates a particle) and the launch (2^20 candidates); with
    // records and rows from a search it also checks the rows against ngb,
    // which k_rows does otherwise
    const bool rows = !mixed && st >= 4 && (st & (st - 1)) == 0;
    A.recs = rows && (c->force_rows || (cands >= 8 * c->n && cands >= ((int64_t)1 << 20)));
    A.verify_rows = A.recs && have && ((uintptr_t)ngb & 15) == 0;
    if (A.verify_rows) {
        // the evaluation checks the rows
    } else if (A.stride % 4 == 0 && ((uintptr_t)ngb & 15) == 0) {
        k_rows4<<<grid_for(n_active * A.stride / 4, 8192), kBlock, 0, c->stream>>>(A, have);
    } else {
        k_rows<<<grid_for(n_active * A.stride, 8192), kBlock, 0, c->stream>>>(A, have);
    }
    c->jsort_ngb = ngb;
    c->jsort_knn = 0;
    // row block summaries for the checks: rows of a power of two entries,
    // written by the first grid check; they pay off on long steps (the
    // first check's extra work against the later checks' savings: 2^26
    // candidates, and at least 8 a particle)
    if (c->csum && c->dev_rounds > 0 && st >= 4 && st <= SIDM_SUM_U && (st & (st - 1)) == 0 &&
        (c->force_rows || (cands >= ((int64_t)1 << 26) && cands >= 8 * c->n)))
        A.csum = c->csum;
    if (c->cfg.periodic) {
        mixed ? run_scatter<true, true>(c, A, n_active, c->stream)
              : run_scatter<true, false>(c, A, n_active, c->stream);
    } else {
        mixed ? run_scatter<false, true>(c, A, n_active, c->stream)
              : run_scatter<false, false>(c, A, n_active, c->stream);
    }
    return hipGetLastError();
}

hipError_t launch_timestep(sidm_ctx *c, int64_t n_active, const int32_t *ngb, const double *h,
                           double *dt_out)
{
    StepArgs A = make_args(c, nullptr, ngb, h, nullptr, 0, 0, nullptr);
    // the rows the scattering step made from the same ngb, if nothing ran since
    if (ngb && c->jsort_ngb == ngb) A.jsort = c->jsort;
    phase_begin(c, PH_TIMESTEP);
    const int k = A.k;
    if (k <= 64 && (k & (k - 1)) == 0) {
        const int64_t lanes = n_active * (k < 4 ? 1 : k / 4);
        if (c->cfg.xsec == SIDM_XSEC_CONST) {
            // velocity records when the gathers they save outweigh writing
            // one for every particle (at least 8 candidates a particle) and
            // the launch (2^20 candidates)
            const int64_t cands = n_active * k;
            if (c->force_rows || (cands >= 8 * c->n && cands >= ((int64_t)1 << 20))) {
                A.vaos = (const double4 *)c->phase;
                k_vel_aos<<<grid_for(2 * c->n, 8192), kBlock, 0, c->stream>>>(c->n, c->vxs, c->vys,
                                                                               c->vzs, (double2 *)c->phase);
                k_timestep_group<true, true><<<grid_for(lanes, 65536), kBlock, 0, c->stream>>>(
                    A, c->cfg.c_sidm, dt_out);
            } else {
                k_timestep_group<true, false><<<grid_for(lanes, 65536), kBlock, 0, c->stream>>>(
                    A, c->cfg.c_sidm, dt_out);
            }
        }
        else
            k_timestep_group<false, false><<<grid_for(lanes, 65536), kBlock, 0, c->stream>>>(
                A, c->cfg.c_sidm, dt_out);
    }
    else
        k_timestep<<<grid_for(n_active), kBlock, 0, c->stream>>>(A, c->cfg.c_sidm, dt_out);
    phase_end(c, PH_TIMESTEP);
    return hipGetLastError();
}

hipError_t launch_scatter_overlap(sidm_ctx *c, sidm_particles *p, int64_t n_active,
                                  int32_t max_ngb, const int32_t *ngb,
                                  const int32_t *count, const double *dt, uint64_t seed,
                                  uint32_t step, uint32_t *cand_info)
{
    StepArgs A = make_args(c, p, ngb, nullptr, dt, seed, step, cand_info);
    A.stride = max_ngb; A.cnt = count;
    if (c->cfg.periodic) run_scatter<true, false, true>(c, A, n_active, c->stream);
    else run_scatter<false, false, true>(c, A, n_active, c->stream);
    return hipGetLastError();
}

hipError_t launch_timestep_overlap(sidm_ctx *c, int64_t n_active, int32_t max_ngb, const int32_t *ngb, const int32_t *count,
                                   double *dt_out)
{
    StepArgs A = make_args(c, nullptr, ngb, nullptr, nullptr, 0, 0, nullptr);
    A.stride = max_ngb; A.cnt = count;
    phase_begin(c, PH_TIMESTEP);
    k_timestep_overlap<<<grid_for(n_active * kTeamT), kBlock, 0, c->stream>>>(A, c->cfg.c_sidm,
                                                                             dt_out);
    phase_end(c, PH_TIMESTEP);
    return hipGetLastError();
}
