// Exact N_ngb-nearest-neighbour search of the active particles (paper sec. 4.2
// and 4.5: h_i is set so that about N_ngb neighbours lie inside the kernel;
// here exactly N_ngb, ties broken by particle ID, h_i = distance of the next).
//
// Two kernels per batch of targets, over the bucket tree (leaves of SIDM_LEAF
// Morton-consecutive particles, SIDM_TREE_FAN-ary parents):
//
//  k_knn_list  one lane per target.  A valid upper bound T on r^2 of the
//              (N_ngb+1)-th neighbour comes from the target's window of
//              Morton-order neighbours: the window's (N_ngb+1)-th smallest r^2,
//              bracketed in FP32 rounded up, so the bound never falls below the
//              exact value.  The wavefront then walks the tree level by level
//              against the box enclosing all its targets' spheres (64 children
//              tested per round, one coalesced load), and each lane keeps the
//              leaves that meet its own sphere.
//
//  k_knn_team  a team of 16 lanes per target, four targets per wavefront.  The
//              team loads the gaps of its whole leaf list at once and takes the
//              leaves nearest first until the nearest left lies beyond the
//              current radius; a leaf's particles are tested 16 at a time
//              (coalesced) and those within the radius are appended to a short
//              LDS list.  When the list fills it is sorted (register bitonic
//              network, E keys per lane) and cut back to N_ngb+1, which
//              tightens the radius.  A target whose list overflowed walks the
//              tree from the root instead (same loop).
//
// Pruning is exact-conservative: a box gap is computed with the same rounded
// operations as a particle separation, and rounding is monotone, so no particle
// with r^2 <= the radius is ever skipped.  The result is the definition:
// the N_ngb smallest (r^2, id) among all other particles, in that order.
#include "sidm_internal.h"

namespace {

struct KnnArgs {
    const double *xs, *ys, *zs;
    const uint32_t *ids;
    const int32_t *perm;
    const double *nodes;
    const int32_t *tlist, *slot;
    const int32_t *nt_dev;
    int32_t *ngb;
    double *h;
    unsigned int *derr;
    int32_t *list;       // [batch][SIDM_KNN_LMAX] leaf lists
    int32_t *nl;         // [batch] list length, -1 on overflow
    double *tb;          // [batch] radius bound from the window
    TreeLevels lv;
    int64_t n, batch;
    int k;
    double box;
};

constexpr int32_t kIdxMask = (1 << SIDM_LEVEL_SHIFT) - 1;

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
    const double *nb = nodes + g * 6;
    const double lx = nb[0], ly = nb[1], lz = nb[2], hx = nb[3], hy = nb[4], hz = nb[5];
    if (!(lx <= hx)) return INFINITY;
    double gx = axis_gap<PERIODIC>(lx, hx, px, box);
    double gy = axis_gap<PERIODIC>(ly, hy, py, box);
    double gz = axis_gap<PERIODIC>(lz, hz, pz, box);
    return (gx * gx + gy * gy) + gz * gz;
}

// squared gap to a box held in registers; +inf for an empty box
template <bool PERIODIC>
__device__ __forceinline__ double box_gap2(const double *bx, double px, double py, double pz, double box)
{
    if (!(bx[0] <= bx[3])) return INFINITY;
    double gx = axis_gap<PERIODIC>(bx[0], bx[3], px, box);
    double gy = axis_gap<PERIODIC>(bx[1], bx[4], py, box);
    double gz = axis_gap<PERIODIC>(bx[2], bx[5], pz, box);
    return (gx * gx + gy * gy) + gz * gz;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// branch-free minimum-image separation^2, identical rounding to sep2<>
template <bool PERIODIC>
__device__ __forceinline__ double sep2_sel(double xi, double yi, double zi, double xj, double yj,
                                           double zj, double box)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    if (PERIODIC) {
        const double half = 0.5 * box;
        dx = dx >= half ? dx - box : (dx < -half ? dx + box : dx);
        dy = dy >= half ? dy - box : (dy < -half ? dy + box : dy);
        dz = dz >= half ? dz - box : (dz < -half ? dz + box : dz);
    }
    return (dx * dx + dy * dy) + dz * dz;
}

// Morton-order window of W other particles around sorted index i
template <int W>
__device__ __forceinline__ void seed_window(int64_t i, int64_t n, int64_t &w0, int64_t &w1)
{
    w0 = i - W / 2;
    if (w0 + W + 1 > n) w0 = n - (W + 1);
    if (w0 < 0) w0 = 0;
    w1 = w0 + W + 1 < n ? w0 + W + 1 : n;
}

__device__ __forceinline__ void cswap(double &ga, int32_t &ia, double &gb, int32_t &ib)
{
    const bool sw = gb < ga;
    const double g = sw ? gb : ga;
    gb = sw ? ga : gb;
    ga = g;
    const int32_t t = sw ? ib : ia;
    ib = sw ? ia : ib;
    ia = t;
}

// ascending sort of 8 (gap, id) pairs: Batcher's odd-even merge network
__device__ __forceinline__ void sort8(double (&g)[8], int32_t (&id)[8])
{
    cswap(g[0], id[0], g[1], id[1]); cswap(g[2], id[2], g[3], id[3]);
    cswap(g[4], id[4], g[5], id[5]); cswap(g[6], id[6], g[7], id[7]);
    cswap(g[0], id[0], g[2], id[2]); cswap(g[1], id[1], g[3], id[3]);
    cswap(g[4], id[4], g[6], id[6]); cswap(g[5], id[5], g[7], id[7]);
    cswap(g[1], id[1], g[2], id[2]); cswap(g[5], id[5], g[6], id[6]);
    cswap(g[0], id[0], g[4], id[4]); cswap(g[1], id[1], g[5], id[5]);
    cswap(g[2], id[2], g[6], id[6]); cswap(g[3], id[3], g[7], id[7]);
    cswap(g[2], id[2], g[4], id[4]); cswap(g[3], id[3], g[5], id[5]);
    cswap(g[1], id[1], g[2], id[2]); cswap(g[3], id[3], g[4], id[4]);
    cswap(g[5], id[5], g[6], id[6]);
}

// Upper bound on the K1-th smallest r^2 among the other particles of the
// Morton-order window [w0, w0 + W], bracketed in FP32 with values rounded up
// (so no count exceeds the exact one); +inf if fewer than K1 fit in FP32.
template <bool PERIODIC, int W>
__device__ __forceinline__ double window_bound(const KnnArgs &A, int64_t i, int64_t w0, double px,
                                               double py, double pz, int K1)
{
    float r2f[W + 1];
    float lo = INFINITY, hi = 0.0f;
#pragma unroll
    for (int t = 0; t <= W; ++t) {
        const int64_t j = w0 + t;
        float v = INFINITY;
        if (j < A.n && j != i)
            v = __double2float_ru(sep2_sel<PERIODIC>(px, py, pz, A.xs[j], A.ys[j], A.zs[j], A.box));
        r2f[t] = v;
        if (v < INFINITY) { lo = fminf(lo, v); hi = fmaxf(hi, v); }
    }
    int c_lo = 0, c_hi = 0;
#pragma unroll
    for (int t = 0; t <= W; ++t) { c_lo += r2f[t] <= lo; c_hi += r2f[t] <= hi; }
    if (c_hi < K1) return INFINITY;
    if (c_lo >= K1) return (double)lo;
    for (int it = 0; it < 12; ++it) {
        const uint32_t bl = __float_as_uint(lo), bh = __float_as_uint(hi);
        if (bh - bl <= 1) break;
        const float mid = __uint_as_float(bl + ((bh - bl) >> 1));
        int c = 0;
#pragma unroll
        for (int t = 0; t <= W; ++t) c += r2f[t] <= mid;
        if (c >= K1) hi = mid; else lo = mid;
    }
    return (double)hi;
}

// ---------------------------------------------------------------------------
// Kernel A: radius bound and per-target leaf list (one lane per target)
// ---------------------------------------------------------------------------
constexpr int kStackA = SIDM_MAX_LEVELS * (SIDM_TREE_FAN - 1) + 1;

constexpr int kFront = 512;               // frontier capacity of the level walk

__device__ __forceinline__ double wave_min(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// does [lo, hi] (or a periodic image of it) meet [glo, ghi]?
template <bool PERIODIC>
__device__ __forceinline__ bool interval_meets(double lo, double hi, double glo, double ghi, double box)
{
    bool m = hi >= glo && lo <= ghi;
    if (PERIODIC) m = m || (hi - box >= glo && lo - box <= ghi) || (hi + box >= glo && lo + box <= ghi);
    return m;
}

template <bool PERIODIC, int W>
__global__ __launch_bounds__(64) void k_knn_list(KnnArgs A, int64_t base)
{
    __shared__ int32_t s_fr[2][kFront];
    __shared__ double s_hit[64 * 6];
    const int nt = *A.nt_dev;
    const int lane = threadIdx.x;
    const int64_t bb = (int64_t)blockIdx.x * 64 + lane;
    const int64_t b = base + bb;
    const bool valid = b < nt && bb < A.batch;
    if (!__any(valid)) return;
    const int32_t i = A.tlist[valid ? b : base + (int64_t)blockIdx.x * 64];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const double box = A.box;
    const int64_t n = A.n;
    const int K1 = A.k + 1;

    // bound: the smaller of two one-sided windows' K1-th smallest r^2 (the
    // W Morton-order particles before and after the target), so a target at a
    // jump of the curve still gets the bound of its compact side
    const int64_t wmax = n - (W + 1) > 0 ? n - (W + 1) : 0;
    const int64_t wl = i - W < 0 ? 0 : (i - W > wmax ? wmax : i - W);
    const int64_t wr = i > wmax ? wmax : i;
    const double T = fmin(window_bound<PERIODIC, W>(A, i, wl, px, py, pz, K1),
                          window_bound<PERIODIC, W>(A, i, wr, px, py, pz, K1));

    // group box: every lane's sphere, padded far beyond rounding, so a box a
    // lane needs always meets it
    const double R = sqrt(T) * (1.0 + 1e-9) + (fabs(px) + fabs(py) + fabs(pz) + box) * 1e-14;
    const double gxl = wave_min(valid ? px - R : INFINITY), gxh = wave_max(valid ? px + R : -INFINITY);
    const double gyl = wave_min(valid ? py - R : INFINITY), gyh = wave_max(valid ? py + R : -INFINITY);
    const double gzl = wave_min(valid ? pz - R : INFINITY), gzh = wave_max(valid ? pz + R : -INFINITY);

    // level-synchronous walk: every round tests up to 64 children (one per
    // lane, one coalesced load); surviving internal nodes form the next
    // frontier, surviving leaves are offered to each lane's own sphere
    int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
    int nl = 0;
    bool ovf = false, wave_ovf = false;
    int cur = 0, fn = 1;
    s_fr[0][0] = 0;                                   // the root (top level, index 0)
    for (int lvl = A.lv.nlev - 1; lvl > 0 && !wave_ovf; --lvl) {
        const int cl = lvl - 1;
        const int64_t ccnt = A.lv.cnt[cl], coff = A.lv.off[cl];
        int nxt = 0;
        const int total = fn * SIDM_TREE_FAN;
        for (int c0 = 0; c0 < total; c0 += 64) {
            const int t = c0 + lane;
            bool hit = false;
            int64_t q = 0;
            double bx[6];
            wave_sync();
            if (t < total) {
                q = (int64_t)s_fr[cur][t / SIDM_TREE_FAN] * SIDM_TREE_FAN + t % SIDM_TREE_FAN;
                if (q < ccnt) {
                    const double *nb = A.nodes + (coff + q) * 6;
#pragma unroll
                    for (int d = 0; d < 6; ++d) bx[d] = nb[d];
                    hit = bx[0] <= bx[3] && interval_meets<PERIODIC>(bx[0], bx[3], gxl, gxh, box) &&
                          interval_meets<PERIODIC>(bx[1], bx[4], gyl, gyh, box) &&
                          interval_meets<PERIODIC>(bx[2], bx[5], gzl, gzh, box);
                }
            }
            const uint64_t m = __ballot(hit);
            const int rank = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            const int nh = __popcll(m);
            if (cl > 0) {
                if (nxt + nh > kFront) { wave_ovf = true; break; }
                if (hit) s_fr[cur ^ 1][nxt + rank] = (int32_t)q;
                nxt += nh;
            } else {
                // leaves: stage the hit boxes, then each lane keeps the ones
                // within its own sphere
                if (hit) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) s_hit[rank * 6 + d] = bx[d];
                    s_fr[cur ^ 1][rank] = (int32_t)q;
                }
                wave_sync();
                for (int h = 0; h < nh; ++h) {
                    const double g = box_gap2<PERIODIC>(s_hit + h * 6, px, py, pz, box);
                    if (valid && g <= T) {
                        if (nl < SIDM_KNN_LMAX) lst[nl++] = s_fr[cur ^ 1][h];
                        else ovf = true;
                    }
                }
            }
        }
        cur ^= 1;
        fn = nxt;
    }
    if (!valid) return;
    A.nl[bb] = (ovf || wave_ovf) ? -1 : nl;
    A.tb[bb] = T;
}

// ---------------------------------------------------------------------------
// Kernel B: exact selection by a 16-lane team per target
// ---------------------------------------------------------------------------
// key order (r^2, id): a < b
__device__ __forceinline__ bool key_lt(double ra, uint32_t ia, double rb, uint32_t ib)
{
    return ra < rb || (ra == rb && ia < ib);
}

// One compare-exchange stage (k = 2^LK, distance d = 2^LD) of an ascending
// bitonic sort of 16*E keys held E per lane (lane tl holds keys tl*E ..
// tl*E+E-1) across a team of 16 lanes.
template <int E, int LK, int LD>
__device__ __forceinline__ void bitonic_stage(double (&r)[E], uint32_t (&id)[E], int32_t (&jj)[E], int tl)
{
    constexpr int k = 1 << LK, d = 1 << LD;
    if constexpr (d < E) {
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const int bq = a ^ d;
            if (bq > a) {
                const bool up = (((tl * E + a) & k) == 0);
                const bool gt = key_lt(r[bq], id[bq], r[a], id[a]);
                const bool sw = gt == up;
                const double ra = r[a], rb = r[bq];
                const uint32_t ia = id[a], ib = id[bq];
                const int32_t ja = jj[a], jb = jj[bq];
                r[a] = sw ? rb : ra; r[bq] = sw ? ra : rb;
                id[a] = sw ? ib : ia; id[bq] = sw ? ia : ib;
                jj[a] = sw ? jb : ja; jj[bq] = sw ? ja : jb;
            }
        }
    } else {
        constexpr int ld = d / E;
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const double orr = __shfl_xor(r[a], ld);
            const uint32_t oid = (uint32_t)__shfl_xor((int)id[a], ld);
            const int32_t oj = __shfl_xor(jj[a], ld);
            const bool up = (((tl * E + a) & k) == 0);
            const bool lower = (tl & ld) == 0;
            const bool take = (lower == up) ? key_lt(orr, oid, r[a], id[a])
                                            : key_lt(r[a], id[a], orr, oid);
            r[a] = take ? orr : r[a];
            id[a] = take ? oid : id[a];
            jj[a] = take ? oj : jj[a];
        }
    }
}

template <int E, int LK, int LD>
__device__ __forceinline__ void bitonic_merge_steps(double (&r)[E], uint32_t (&id)[E], int32_t (&jj)[E], int tl)
{
    bitonic_stage<E, LK, LD>(r, id, jj, tl);
    if constexpr (LD > 0) bitonic_merge_steps<E, LK, LD - 1>(r, id, jj, tl);
}

template <int E, int LK, int LOGN>
__device__ __forceinline__ void bitonic_levels(double (&r)[E], uint32_t (&id)[E], int32_t (&jj)[E], int tl)
{
    bitonic_merge_steps<E, LK, LK - 1>(r, id, jj, tl);
    if constexpr (LK < LOGN) bitonic_levels<E, LK + 1, LOGN>(r, id, jj, tl);
}

template <int E>
__device__ __forceinline__ void team_sort(double (&r)[E], uint32_t (&id)[E], int32_t (&jj)[E], int tl)
{
    constexpr int LOGN = (E == 4) ? 6 : 7;     // 16*E keys
    bitonic_levels<E, 1, LOGN>(r, id, jj, tl);
}

constexpr int kStackB = 7 * 9 + 1;       // deepest walk: 10 levels (n < 2^31) of 8-ary nodes

template <bool PERIODIC, int E>
__global__ __launch_bounds__(256) void k_knn_team(KnnArgs A, int64_t base)
{
    constexpr int N = 16 * E;                 // list capacity
    __shared__ int32_t s_stack[16][kStackB];  // only the overflow walk uses it
    __shared__ double s_r2[16][N];
    __shared__ uint32_t s_id[16][N];
    __shared__ int32_t s_j[16][N];

    const int team = threadIdx.x >> 4, tl = threadIdx.x & 15;
    const int wteam = team & 3;               // team within the wavefront
    const int nt = *A.nt_dev;
    const int64_t bb = (int64_t)blockIdx.x * 16 + team;
    const int64_t b = base + bb;
    if (!(b < nt && bb < A.batch)) return;    // whole team
    const int32_t i = A.tlist[b];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const double box = A.box;
    const int64_t n = A.n;
    const int K1 = A.k + 1;
    const uint32_t *__restrict__ ids = A.ids;
    double *L_r2 = s_r2[team];
    uint32_t *L_id = s_id[team];
    int32_t *L_j = s_j[team];
    int32_t *stk = s_stack[team];

    // leaves come from the target's list (nearest first), read 16 at a time
    // with one lane per leaf box; a target whose list overflowed walks the
    // tree from the root with a stack (packed (level << SIDM_LEVEL_SHIFT) | index)
    const int nl = A.nl[bb];
    const int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
    const bool walk = nl < 0;
    int sp = 0;
    if (walk) {
        if (tl == 0) stk[0] = (A.lv.nlev - 1) << SIDM_LEVEL_SHIFT;
        sp = 1;
    }
    // gaps of the whole list (one round of loads); leaves are then taken
    // nearest first, and the walk ends when the nearest left is beyond T
    constexpr int kPer = (SIDM_KNN_LMAX + 15) / 16;
    double lg[kPer];
    int32_t lf[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int t = q * 16 + tl;
        lf[q] = (!walk && t < nl) ? lst[t] : -1;
        lg[q] = lf[q] >= 0 ? node_gap2<PERIODIC>(A.nodes, lf[q], px, py, pz, box) : INFINITY;
    }

    double T = A.tb[bb];
    int count = 0;
    double r[E];
    uint32_t id[E];
    int32_t jj[E];
    const uint64_t below = (tl == 0) ? 0ull : ((1ull << tl) - 1ull);
    int64_t cur_s0 = 0;
    int cur_m = 0, cur_off = 0;
    double q1x = 0, q1y = 0, q1z = 0, q0x = 0, q0y = 0, q0z = 0;
    bool done = false, finished = false;
    wave_sync();
    while (true) {
        // the teams of a wavefront sort together whenever one of them must
        // (sorting is idempotent), so the network runs once for all four
        const bool want = !finished && (done || count + 16 > N);
        if (__any(want) && !finished) {
            // sort the list, keep the best K1, tighten the radius
            wave_sync();
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int e = tl * E + q;
                if (e < count) { r[q] = L_r2[e]; id[q] = L_id[e]; jj[q] = L_j[e]; }
                else { r[q] = INFINITY; id[q] = 0xffffffffu; jj[q] = -1; }
            }
            team_sort<E>(r, id, jj, tl);
            wave_sync();
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int e = tl * E + q;
                if (e < K1) { L_r2[e] = r[q]; L_id[e] = id[q]; L_j[e] = jj[q]; }
            }
            wave_sync();
            if (count >= K1) T = L_r2[K1 - 1];
            count = count < K1 ? count : K1;
            if (done) finished = true;
        }
        if (__all(finished)) break;
        if (finished) continue;
        if (cur_off >= cur_m) {
            // next leaf within the radius
            cur_m = 0;
            cur_off = 0;
            while (true) {
                if (!walk) {
                    // team argmin over (gap, lane, slot)
                    double bg = INFINITY;
                    int bq = 0;
#pragma unroll
                    for (int q = 0; q < kPer; ++q)
                        if (lg[q] < bg) { bg = lg[q]; bq = q; }
                    int bl = tl;
                    for (int off = 1; off < 16; off <<= 1) {
                        const double og = __shfl_xor(bg, off);
                        const int ol = __shfl_xor(bl, off), oq = __shfl_xor(bq, off);
                        if (og < bg || (og == bg && ol < bl)) { bg = og; bl = ol; bq = oq; }
                    }
                    if (!(bg <= T)) break;
                    int32_t leaf = -1;
#pragma unroll
                    for (int q = 0; q < kPer; ++q)
                        if (q == bq) leaf = lf[q];
                    leaf = __shfl(leaf, bl, 16);
                    if (tl == bl) {
#pragma unroll
                        for (int q = 0; q < kPer; ++q)
                            if (q == bq) lg[q] = INFINITY;
                    }
                    cur_s0 = (int64_t)leaf * SIDM_LEAF;
                } else {
                    if (sp == 0) break;
                    --sp;
                    const int32_t e = stk[sp];
                    const int lvl = e >> SIDM_LEVEL_SHIFT;
                    const int64_t q = e & kIdxMask;
                    const double d2 = node_gap2<PERIODIC>(A.nodes, A.lv.off[lvl] + q, px, py, pz, box);
                    if (!(d2 <= T)) continue;
                    if (lvl > 0) {
                        // push the children within the radius, nearest on top
                        const int cl = lvl - 1;
                        const int64_t cq = q * SIDM_TREE_FAN + tl;
                        double gc = INFINITY;
                        if (tl < SIDM_TREE_FAN && cq < A.lv.cnt[cl])
                            gc = node_gap2<PERIODIC>(A.nodes, A.lv.off[cl] + cq, px, py, pz, box);
                        const bool ok = gc <= T && gc < INFINITY;
                        int rank = 0;
#pragma unroll
                        for (int s2 = 0; s2 < SIDM_TREE_FAN; ++s2) {
                            const double go = __shfl(gc, s2, 16);
                            const bool oo = go <= T && go < INFINITY;
                            rank += oo && (go < gc || (go == gc && s2 < tl));
                        }
                        const uint64_t m = (__ballot(ok) >> (wteam * 16)) & 0xffffull;
                        const int np = __popcll(m);
                        wave_sync();
                        if (ok) stk[sp + np - 1 - rank] = (cl << SIDM_LEVEL_SHIFT) | (int32_t)cq;
                        sp += np;
                        wave_sync();
                        continue;
                    }
                    cur_s0 = q * SIDM_LEAF;
                }
                cur_m = (int)((n - cur_s0) < SIDM_LEAF ? (n - cur_s0) : SIDM_LEAF);
                // both 16-particle halves of the leaf in one round of loads
                const int64_t j0 = cur_s0 + (tl < cur_m ? tl : 0);
                const int64_t j1 = cur_s0 + (tl + 16 < cur_m ? tl + 16 : 0);
                q0x = A.xs[j0]; q0y = A.ys[j0]; q0z = A.zs[j0];
                q1x = A.xs[j1]; q1y = A.ys[j1]; q1z = A.zs[j1];
                break;
            }
            if (cur_m == 0) { done = true; continue; }
        }
        // 16 particles of the current leaf
        const int c = cur_off + tl;
        const int64_t j = cur_s0 + c;
        const bool first = cur_off == 0;
        bool pass = false;
        double r2 = 0.0;
        if (c < cur_m) {
            r2 = sep2_sel<PERIODIC>(px, py, pz, first ? q0x : q1x, first ? q0y : q1y,
                                    first ? q0z : q1z, box);
            pass = r2 <= T && j != i;
        }
        const uint64_t mask = (__ballot(pass) >> (wteam * 16)) & 0xffffull;
        if (pass) {
            const int pos = count + __popcll(mask & below);
            L_r2[pos] = r2;
            L_id[pos] = ids[j];
            L_j[pos] = (int32_t)j;
        }
        count += __popcll(mask);
        cur_off += 16;
    }

    const int32_t a = A.slot[b];
    if (count < K1) {                          // cannot happen: T bounds K1 window particles
        if (tl == 0) atomicOr(A.derr, DERR_COUNT);
        return;
    }
    if (tl == 0) A.h[a] = sqrt(T);
    int32_t *out = A.ngb + (int64_t)a * A.k;
    for (int e = tl; e < A.k; e += 16) out[e] = A.perm[L_j[e]];
}

template <bool P, int E>
void launch_batches(const KnnArgs &A0, int64_t n_active, int64_t nb_cap, hipStream_t s)
{
    for (int64_t base = 0; base < n_active; base += nb_cap) {
        KnnArgs A = A0;
        A.batch = (n_active - base) < nb_cap ? (n_active - base) : nb_cap;
        k_knn_list<P, 16 * E><<<(unsigned)((A.batch + 63) / 64), 64, 0, s>>>(A, base);
        k_knn_team<P, E><<<(unsigned)((A.batch + 15) / 16), 256, 0, s>>>(A, base);
    }
}

}  // namespace

hipError_t launch_knn(sidm_ctx *c, int64_t n_active, int32_t *ngb, double *h)
{
    KnnArgs A;
    A.xs = c->xs; A.ys = c->ys; A.zs = c->zs;
    A.ids = c->ids; A.perm = c->perm; A.nodes = c->nodes;
    A.tlist = c->tlist; A.slot = c->slot; A.nt_dev = c->nt_dev;
    A.ngb = ngb; A.h = h; A.derr = c->derr;
    A.list = c->knn_list; A.nl = c->knn_nl; A.tb = c->knn_tb;
    A.lv = c->lv;
    A.n = c->n; A.k = c->cfg.n_ngb; A.box = c->cfg.box; A.batch = 0;
    const bool per = c->cfg.periodic != 0;
    const int k1 = A.k + 1;
    phase_begin(c, PH_KNN);
    if (k1 + 16 <= 64) {
        per ? launch_batches<true, 4>(A, n_active, c->knn_batch, c->stream)
            : launch_batches<false, 4>(A, n_active, c->knn_batch, c->stream);
    } else {
        per ? launch_batches<true, 8>(A, n_active, c->knn_batch, c->stream)
            : launch_batches<false, 8>(A, n_active, c->knn_batch, c->stream);
    }
    phase_end(c, PH_KNN);
    return hipGetLastError();
}
