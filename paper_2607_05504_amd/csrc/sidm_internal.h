// Internal declarations of the gfx950 SIDM library: context layout, device
// helpers shared by the kernels, and the host-side launchers each .hip file
// provides.  Not part of the public ABI (include/sidm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sidm.h"

#define SIDM_PI 3.14159265358979323846
#define SIDM_LEAF 32            // particles per tree leaf (consecutive in Morton order)
#define SIDM_SUB 8              // particles per sub-bucket of a leaf (its own box, for the search)
#define SIDM_SORT_TILE 2048     // keys per radix-sort workgroup (256 threads x 8)
#define SIDM_SCAN_TILE 1024     // elements per compaction workgroup
#define SIDM_TIMING_RING 256    // timed launches per phase between two reads
#define SIDM_PHASES 7           // timed phases (PH_* below)
#define SIDM_KNN_LMAX 96        // leaves per target list (longer lists walk the tree instead)
#define SIDM_KNN_BATCH (1 << 22)  // targets per neighbour-search batch

// device-side error bits (latched, reported by sidm_sync)
#define DERR_INDEX 1u           // an index outside [0, n)
#define DERR_DUPLICATE 2u       // an active particle listed twice
#define DERR_OVERFLOW 4u        // accepted-candidate list overflow
#define DERR_COUNT 8u           // fewer than n_ngb + 1 candidates found
#define DERR_STALL 16u          // a resolution pass decided nothing (cannot happen)
#define DERR_NGB_OVERFLOW 32u   // an overlap row longer than its buffer
#define DERR_BAD_H 64u          // a smoothing length that is not > 0 and finite
#define DERR_HISTORY 128u       // the scatter histories of a step outgrew their buffer

#define SIDM_TREE_FAN 8         // children per internal tree node
#define SIDM_MAX_LEVELS 12
#define SIDM_LEVEL_SHIFT 27     // packed node id: (level << 27) | index within level

// Level layout of the bucket tree: level 0 holds the leaves, level l+1 the
// parents of groups of SIDM_TREE_FAN consecutive level-l nodes; the top level
// has one node.  Node (l, q) is stored at nodes[off[l] + q].
struct TreeLevels {
    int32_t nlev;
    int64_t off[SIDM_MAX_LEVELS];
    int64_t cnt[SIDM_MAX_LEVELS];
};

inline TreeLevels tree_levels(int64_t n)
{
    TreeLevels t = {};
    int64_t c = (n + SIDM_LEAF - 1) / SIDM_LEAF, off = 0;
    if (c < 1) c = 1;
    t.nlev = 0;
    while (true) {
        t.off[t.nlev] = off;
        t.cnt[t.nlev] = c;
        t.nlev++;
        off += c;
        if (c == 1 && t.nlev > 1) break;
        c = (c + SIDM_TREE_FAN - 1) / SIDM_TREE_FAN;
    }
    return t;
}

inline int64_t tree_node_count(const TreeLevels &t)
{
    return t.off[t.nlev - 1] + t.cnt[t.nlev - 1];
}

struct DevStats {
    unsigned long long n_cand, n_accept0, n_events, n_flagged, n_p_ge_1, n_recheck;
    unsigned long long max_p_bits;      // positive doubles order like their bit patterns
    unsigned int n_passes, n_rounds;
};

// The candidates (i|j) of a step whose turns are replayed in order (accepted
// with the step-start velocities, or found to accept at their turn later),
// kept in structure-of-arrays form.
struct AccList {
    int32_t *i, *j;          // sorted-order particle indices (target, partner)
    int32_t *cand;           // a * stride + s  (caller's active slot and neighbour slot)
    double *u;               // decision draw
    double *W;               // kernel weight W(r_ij, h_i) (positions do not change)
    double *dt;              // timestep of the target
    uint64_t *prio;          // priority word
    uint64_t *idpair;        // (id_i << 32) | id_j
    int32_t *rec;            // its turn's record pair (first record), -1 before its turn
};

// One turn of a listed candidate at one of its two particles: the particle's
// history within the step is the chain of these records, latest first.
struct TurnRecords {
    uint64_t *prio, *idpair; // the candidate's key
    double *vx, *vy, *vz;    // the particle's velocity just before the turn
    int32_t *mem;            // index of the candidate in the list
    int32_t *prev;           // the particle's previous record, -1 if none
    int32_t *part;           // the particle (sorted index)
    uint32_t *info;          // bit 0: kicked; bits 1..7: state before; bits 8..: kick depth after
};

#define SIDM_FLAG_CAP 4096    // candidates whose flagged status a step re-counts at its end

// Block summaries of the candidate rows, for the checks of a small D: the
// rows in the tree's order are cut into blocks of SIDM_SUM_U candidates, and
// each block records the index buckets (SIDM_DBUCKET particles of the sorted
// order each) of its targets and partners.  Sixteen int32 a block: [0..1] a
// 64-bit mask of the buckets base - 32 .. base + 31, [2] base (the first
// target's bucket), [3] the number of other buckets (-1: too many to list,
// the block is always scanned), [4..15] those buckets.
#define SIDM_SUM_U 1024
#define SIDM_SUM_WORDS 16
#define SIDM_SUM_OUT 12
#define SIDM_DBUCKET_SHIFT 8
// words of the bucket bitmap for n particles
inline int64_t bucket_words(int64_t n) { return ((n >> SIDM_DBUCKET_SHIFT) + 1 + 31) / 32; }

struct sidm_ctx {
    sidm_config cfg;
    int64_t cap_n, cap_active, cap_acc, cap_rec;
    int device;
    hipStream_t stream;
    char err[512];

    // snapshot of the particles in Morton order
    int64_t n;
    int tree_ok;
    int64_t sorted_n;        // particles of the last full sort (0: none)
    int has_mass;
    double m_scalar;         // particle mass when no per-particle array is given
    double *xs, *ys, *zs, *vxs, *vys, *vzs, *ms;
    uint32_t *ids;
    uint8_t *sts;
    double *rec;             // [cap_n * 8] the caller's particles as 64-byte records
    int32_t *perm;           // sorted -> caller index
    int32_t *inv;            // caller -> sorted index

    // radix sort scratch
    uint64_t *key0, *key1;
    int32_t *val0, *val1;
    uint32_t *hist;          // [256][n_sort_blocks]
    uint32_t *dtot;          // [6][256] digit totals of every pass
    unsigned long long *bounds;   // ordered-u64 encodings of min x,y,z / max x,y,z

    // bucket tree: leaves of SIDM_LEAF consecutive particles (level 0) and
    // levels of SIDM_TREE_FAN-ary parents above them, boxes level after level
    TreeLevels lv;
    double *nodes;           // [nodes][6]  lo x,y,z, hi x,y,z
    float *sbox;             // [leaves * SIDM_LEAF / SIDM_SUB][8]  sub-bucket boxes, FP32 rounded
                             // outward: lo x,y,z, 0, hi x,y,z, 0
    // mixed form only: FP32 offsets of each particle from its leaf's box
    // centre 0.5 (lo + hi), the centre itself rounded as that FP64 expression
    float *xo, *yo, *zo;

    // neighbour search: per-target leaf lists, processed in batches of knn_batch
    int64_t knn_batch;
    char *phase;             // buffer of the tree build's and the search's temporaries
    int32_t *knn_list;       // [knn_batch][SIDM_KNN_LMAX]   (in phase)
    // the rows in the tree's order: jsort[b * n_ngb + s] = sorted index of
    // neighbour s of the b-th target in Morton order (-1 for an index out of
    // range).  sidm_find_ngb writes them beside ngb; sidm_scatter_step checks
    // them against its ngb (translating any entry that differs), and
    // sidm_pair_timestep reads them given the same ngb while nothing else ran
    int32_t *jsort;          // [cap_active * n_ngb]
    const int32_t *jsort_ngb;     // the ngb they match, NULL if none
    int jsort_knn;           // they are the last sidm_find_ngb's, for the current mapping
    // per batch, in two sets that alternate between batches (a batch's root
    // walk runs on knn_aux while the next batch is searched)
    int32_t *knn_nl[2];      // [knn_batch]   (in phase)
    int32_t *knn_fb[2];      // [knn_batch] targets of a batch left to the root walk (in phase)
    int32_t *knn_fbn[2];     // [1] their number
    hipStream_t knn_aux;     // default priority
    hipEvent_t knn_ev[2][2]; // [set][0: sub-bucket kernel done, 1: root walk done]
    double *knn_tb[2];       // [knn_batch]   (in phase)

    // active set in Morton order
    int32_t *flag;           // [cap_n] caller slot of an active particle, or -1
    int32_t *tlist;          // [cap_active] sorted index of the b-th active particle
    int32_t *slot;           // [cap_active] its position in the caller's active list
    int32_t *blk;            // compaction block counts / offsets
    int32_t *nt_dev;         // number of compacted targets
    int map_valid;           // the arrays above hold the mapping of map_n targets
    int64_t map_n;           //   made since the last tree build (reusable: active == NULL)

    // the turns of the step in (priority, id_i, id_j) order
    AccList mem;             // [cap_acc] listed candidates
    int32_t *mmark;          // [cap_acc] 1 while a listed candidate is marked for replay
    int32_t *wl[2];          // [cap_acc] pass work lists (indices into mem)
    int32_t *plist;          // [2 cap_acc] particles whose history a re-round rewinds
    TurnRecords trec;        // [cap_rec] turn records, in pairs (one per particle of a turn)
    int32_t *rfree;          // [cap_rec / 2] record pairs a rewind freed
    int32_t *head;           // [cap_n] latest turn record of each particle, -1 if none
    unsigned long long *tmin;     // [cap_n] smallest priority a re-round replays, ~0 if none
    uint32_t *dbits;         // [cap_n / 32] bit per sorted index: the particle is in D
    uint32_t *bbits;         // [cap_n / 2^(5 + SIDM_DBUCKET_SHIFT)] bit per index bucket: holds a particle of D
    int32_t *csum;           // [cap_active * n_ngb / SIDM_SUM_U][SIDM_SUM_WORDS] row block summaries, or NULL
    int32_t *flist;          // [2 SIDM_FLAG_CAP] (target, candidate slot) once flagged
    int32_t *acc_count;      // [16] control words (list counts, passes, rounds)
    unsigned long long *claim1[2], *claim2[2];   // [cap_n] per-particle claims
    int dev_rounds;          // rounds run as grid launches before the one-workgroup tail
    int force_rows;          // row block summaries and partner records whatever the sizes (tests)

    DevStats *dstats;
    unsigned int *derr;
    double *xt_w, *xt_s;     // tabulated cross-section nodes [SIDM_XSEC_TABLE_MAX]
    double *xt_lw;           //   and the natural logarithms of their speeds
    // overlap estimator only: every particle's h in Morton order, the largest
    // h below every tree node, and the ghat table
    double *hs, *hmax, *gtab;
    int hs_valid;            // hs holds hs_src gathered for the current tree
    const double *hs_src;
    unsigned long long *adv_min;   // served form: smallest per-pair bound of a step
    // opt-in event timing of the main kernels: up to SIDM_TIMING_RING launches
    // of each phase are bracketed between two sidm_timing_read calls
    int timing;              // mask of the timed phases (bit PH_*)
    hipEvent_t ev[SIDM_PHASES][SIDM_TIMING_RING][2];
    int ev_count[SIDM_PHASES];
    void *dev_base;          // the one device allocation every buffer above lives in
    DevStats *hstats;        // pinned host copy
    unsigned int *herr;
};

// ---------------------------------------------------------------------------
// Device helpers (shared by the kernels of this library)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ordered_u64(double v)
{
    unsigned long long b = __double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_u64(unsigned long long b)
{
    return __longlong_as_double((b >> 63) ? (b & 0x7fffffffffffffffull) : ~b);
}

// Minimum-image separation of one axis: d = x_j - x_i, wrapped once.
template <bool PERIODIC>
__device__ __forceinline__ double axis_sep(double xi, double xj, double box)
{
    double d = xj - xi;
    if (PERIODIC) {
        if (d >= 0.5 * box) d = d - box;
        else if (d < -0.5 * box) d = d + box;
    }
    return d;
}

template <bool PERIODIC>
__device__ __forceinline__ double sep2(double xi, double yi, double zi, double xj, double yj,
                                       double zj, double box)
{
    double dx = axis_sep<PERIODIC>(xi, xj, box);
    double dy = axis_sep<PERIODIC>(yi, yj, box);
    double dz = axis_sep<PERIODIC>(zi, zj, box);
    return (dx * dx + dy * dy) + dz * dz;
}

// gap along one axis between point p and a box [lo, hi], as a particle's
// separation would round (min over the periodic images)
template <bool PERIODIC>
__device__ __forceinline__ double axis_gap(double lo, double hi, double p, double box)
{
    double a = lo - p, b = hi - p;
    double g = a > 0.0 ? a : (b < 0.0 ? -b : 0.0);
    if (PERIODIC) {
        double am = a - box, bm = b - box;   // image shifted by -L
        double gm = am > 0.0 ? am : (bm < 0.0 ? -bm : 0.0);
        double ap = a + box, bp = b + box;   // image shifted by +L
        double gp = ap > 0.0 ? ap : (bp < 0.0 ? -bp : 0.0);
        g = fmin(g, fmin(gm, gp));
    }
    return g;
}

// squared gap to the box stored at nodes[g]; +inf for an empty box
template <bool PERIODIC>
__device__ __forceinline__ double node_gap2(const double *__restrict__ nodes, int64_t g, double px,
                                            double py, double pz, double box)
{
    // branch-free, so that the six bounds are requested together (an early
    // return for an empty box made the compiler wait for lo.x and hi.x first)
    const double *nb = nodes + g * 6;
    const double lx = nb[0], ly = nb[1], lz = nb[2], hx = nb[3], hy = nb[4], hz = nb[5];
    double gx = axis_gap<PERIODIC>(lx, hx, px, box);
    double gy = axis_gap<PERIODIC>(ly, hy, py, box);
    double gz = axis_gap<PERIODIC>(lz, hz, pz, box);
    const double g2 = (gx * gx + gy * gy) + gz * gz;
    return lx <= hx ? g2 : INFINITY;
}

// XCD-aware block order.  The 8 XCDs of an MI355X each have their own L2, and
// a launch deals its workgroups to them round-robin (workgroup b to XCD
// b % 8).  Launched with xcd_grid(g) workgroups, xcd_block maps them so that
// each XCD runs runs of xcd_run(g) consecutive logical blocks (spatially
// close targets share an L2), the runs dealt round-robin so that the XCDs'
// loads stay balanced: runs of g / 64 blocks (at least eight a XCD), from 16
// to SIDM_XCD_RUN.  Returns -1 for the padding workgroups, which must do
// nothing.
#define SIDM_XCDS 8
#define SIDM_XCD_RUN 256
__host__ __device__ inline int64_t xcd_run(int64_t g)
{
    const int64_t r = g / (8 * SIDM_XCDS);
    return r < 16 ? 16 : r > SIDM_XCD_RUN ? SIDM_XCD_RUN : r;
}
inline unsigned xcd_grid(int64_t g)
{
    const int64_t span = (int64_t)SIDM_XCDS * xcd_run(g);
    return (unsigned)((g + span - 1) / span * span);
}
__device__ __forceinline__ int64_t xcd_block(int64_t g)
{
    const int64_t run = xcd_run(g);
    const int64_t b = blockIdx.x;
    const int64_t x = b % SIDM_XCDS, k = b / SIDM_XCDS;     // k-th workgroup on XCD x
    const int64_t logical = (k / run) * (SIDM_XCDS * run) + x * run + k % run;
    return logical < g ? logical : -1;
}

// Grid-stride loops: the logical block of this workgroup, such that the
// workgroups of one XCD (dealt b % 8) take consecutive blocks of each stride
// and the rows they read stay in that XCD's L2.  gridDim.x is a multiple of 8
// (grid8 on the host).
__device__ __forceinline__ int64_t xcd_stride_block()
{
    const int64_t b = blockIdx.x, per = gridDim.x / SIDM_XCDS;
    return (b % SIDM_XCDS) * per + b / SIDM_XCDS;
}
inline int grid8(int64_t g)
{
    return (int)((g + SIDM_XCDS - 1) / SIDM_XCDS * SIDM_XCDS);
}

// Cubic spline kernel W_CS(r, h) with support radius h.
__device__ __forceinline__ double cubic_spline(double r, double h)
{
    double h3 = (h * h) * h;
    double norm = 8.0 / (SIDM_PI * h3);
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

// Tabulated sigma(w)/m over nodes tw[0..n) (increasing): linear in ln w
// between the bracketing nodes (found by bisection; tlw holds the nodes'
// ln w), the end values outside.
__device__ __forceinline__ double xsec_table(double w, const double *tw, const double *tlw,
                                             const double *ts, int n)
{
    if (!(w > tw[0])) return ts[0];
    if (!(w < tw[n - 1])) return ts[n - 1];
    int lo = 0, hi = n - 1;                // tw[lo] <= w < tw[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tw[mid] <= w) lo = mid; else hi = mid;
    }
    const double f = (log(w) - tlw[lo]) / (tlw[hi] - tlw[lo]);
    return ts[lo] + f * (ts[hi] - ts[lo]);
}

__device__ __forceinline__ double xsec_sigma(double w, int xsec, double s0, double w0)
{
    if (xsec == SIDM_XSEC_YUKAWA) {
        double x = w / w0;
        double d = 1.0 + x * x;
        return s0 / (d * d);
    }
    return s0;
}

// g_ij of the overlap estimator: the ghat table (SIDM_OVERLAP_NA+1 rows of
// SIDM_OVERLAP_NR+1) read bilinearly at alpha = min(h_i, h_j)/H,
// rho = r/H, over H^3 (H = h_i + h_j); zero for r >= H
__device__ __forceinline__ double overlap_g(const double *__restrict__ tab, double hi, double hj,
                                            double r)
{
    const double H = hi + hj;
    const double al = (hi < hj ? hi : hj) / H;
    const double rho = r / H;
    if (!(rho < 1.0)) return 0.0;
    const double fa = al * (2.0 * SIDM_OVERLAP_NA), fr = rho * SIDM_OVERLAP_NR;
    int ia = (int)fa, ir = (int)fr;
    if (ia > SIDM_OVERLAP_NA - 1) ia = SIDM_OVERLAP_NA - 1;
    if (ir > SIDM_OVERLAP_NR - 1) ir = SIDM_OVERLAP_NR - 1;
    const double ta = fa - ia, tr = fr - ir;
    const double *t0 = tab + ia * (SIDM_OVERLAP_NR + 1) + ir;
    const double *t1 = t0 + (SIDM_OVERLAP_NR + 1);
    const double g0 = t0[0] + tr * (t0[1] - t0[0]);
    const double g1 = t1[0] + tr * (t1[1] - t1[0]);
    return (g0 + ta * (g1 - g0)) / ((H * H) * H);
}

// overlap_g at r = 0, where the radial weight tr is 0 and only the table's
// first column is read (the same value, bit for bit)
__device__ __forceinline__ double overlap_g0(const double *__restrict__ tab, double hi, double hj)
{
    const double H = hi + hj;
    const double al = (hi < hj ? hi : hj) / H;
    const double fa = al * (2.0 * SIDM_OVERLAP_NA);
    int ia = (int)fa;
    if (ia > SIDM_OVERLAP_NA - 1) ia = SIDM_OVERLAP_NA - 1;
    const double ta = fa - ia;
    const double g0 = tab[ia * (SIDM_OVERLAP_NR + 1)], g1 = tab[(ia + 1) * (SIDM_OVERLAP_NR + 1)];
    return (g0 + ta * (g1 - g0)) / ((H * H) * H);
}

__device__ __forceinline__ double rel_speed(double ax, double ay, double az, double bx,
                                            double by, double bz)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

__device__ __forceinline__ double pair_prob(double m_j, double sig, double w, double W, double dt)
{
    return (((0.5 * m_j) * sig) * w * W) * dt;
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round's two
// products are taken whole (32 x 32 -> 64 bits: one v_mad_u64_u32 each, where
// separate high and low halves cost two quarter-rate multiplies).
struct Philox4 { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    }
    return Philox4{c0, c1, c2, c3};
}

#define PURPOSE_DECIDE 0u
#define PURPOSE_DIR_LO_HI 1u
#define PURPOSE_PRIORITY 2u
#define PURPOSE_DIR_HI_LO 3u

__device__ __forceinline__ Philox4 pair_draw(uint64_t seed, uint32_t step, uint32_t ida,
                                             uint32_t idb, uint32_t purpose)
{
    uint32_t lo = ida < idb ? ida : idb, hi = ida < idb ? idb : ida;
    return philox4x32_10(lo, hi, step, purpose, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ uint64_t direction_word(const Philox4 &x, bool target_is_lower)
{
    return target_is_lower ? ((uint64_t)x.x1 << 32 | x.x0) : ((uint64_t)x.x3 << 32 | x.x2);
}

__device__ __forceinline__ double unit_from_word(uint64_t w)
{
    return (double)(w >> 11) * 0x1.0p-53;
}

// phases timed by sidm_timing
enum { PH_TREE = 0, PH_MAP = 1, PH_KNN = 2, PH_EVAL = 3, PH_RESOLVE = 4, PH_TIMESTEP = 5,
       PH_OVERLAP = 6 };
static_assert((1 << PH_TREE) == SIDM_TIMING_TREE && (1 << PH_KNN) == SIDM_TIMING_KNN &&
                  (1 << PH_OVERLAP) == SIDM_TIMING_OVERLAP && (1 << SIDM_PHASES) - 1 == SIDM_TIMING_ALL,
              "phase bits of sidm_timing_enable");

inline void phase_begin(sidm_ctx *c, int ph)
{
    if (((c->timing >> ph) & 1) && c->ev_count[ph] < SIDM_TIMING_RING)
        (void)hipEventRecord(c->ev[ph][c->ev_count[ph]][0], c->stream);
}
inline void phase_end(sidm_ctx *c, int ph)
{
    if (((c->timing >> ph) & 1) && c->ev_count[ph] < SIDM_TIMING_RING) {
        (void)hipEventRecord(c->ev[ph][c->ev_count[ph]][1], c->stream);
        c->ev_count[ph]++;
    }
}

// ---------------------------------------------------------------------------
// Launchers (host side), one group per .hip file
// ---------------------------------------------------------------------------
// tree.hip
hipError_t launch_build_tree(sidm_ctx *c, const sidm_particles *p);
hipError_t launch_refit_tree(sidm_ctx *c, const sidm_particles *p);
hipError_t launch_map_active(sidm_ctx *c, const int32_t *active, int64_t n_active);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

// FP32 minimum image of an offset already reduced to about [-L, L) (mixed form)
__device__ __forceinline__ float wrap32(float d, float box)
{
    const float half = 0.5f * box;
    return d >= half ? d - box : (d < -half ? d + box : d);
}

// centre of a box stored as lo x,y,z, hi x,y,z (the reference point of the
// FP32 offsets of the mixed form)
__device__ __forceinline__ double box_centre(const double *b, int d)
{
    return 0.5 * (b[d] + b[d + 3]);
}
// knn.hip
hipError_t launch_knn(sidm_ctx *c, int64_t n_active, int32_t *ngb, double *h);
// scatter.hip
hipError_t launch_scatter(sidm_ctx *c, sidm_particles *p, int64_t n_active, const int32_t *ngb,
                          const double *h, const double *dt, uint64_t seed, uint32_t step,
                          uint32_t *cand_info);
hipError_t launch_timestep(sidm_ctx *c, int64_t n_active, const int32_t *ngb, const double *h,
                           double *dt_out);
// (both read every particle's h from the Morton-order copy c->hs)
hipError_t launch_scatter_overlap(sidm_ctx *c, sidm_particles *p, int64_t n_active,
                                  int32_t max_ngb, const int32_t *ngb,
                                  const int32_t *count, const double *dt, uint64_t seed,
                                  uint32_t step, uint32_t *cand_info);
hipError_t launch_timestep_overlap(sidm_ctx *c, int64_t n_active, int32_t max_ngb, const int32_t *ngb, const int32_t *count,
                                   double *dt_out);
// overlap.hip
hipError_t launch_overlap_table(sidm_ctx *c);
hipError_t launch_find_overlap(sidm_ctx *c, double *h_all, const double *h_active,
                               int64_t n_active, int32_t max_ngb, int32_t *ngb, int32_t *count);
hipError_t launch_gather_h(sidm_ctx *c, const double *h_all);
// advance.hip
hipError_t launch_advance(sidm_ctx *c, double *x, double *y, double *z, double *vx, double *vy,
                          double *vz, int64_t n, const double *dt_sidm, int64_t n_active,
                          double dt_cap, double gm, double a, double *dt_next, double *dt_step);
hipError_t launch_drift(sidm_ctx *c, double *x, double *y, double *z, const double *vx,
                        const double *vy, const double *vz, int64_t n, double dt);
