// Exact N_ngb-nearest-neighbour search of the active particles (paper sec. 4.2
// and 4.5: h_i is set so that about N_ngb neighbours lie inside the kernel;
// here exactly N_ngb, ties broken by particle ID, h_i = distance of the next).
//
// Three kernels per batch of targets, over the bucket tree (leaves of
// SIDM_LEAF Morton-consecutive particles, each split into sub-buckets of
// SIDM_SUB with their own boxes; SIDM_TREE_FAN-ary parents):
//
//  k_knn_list   four (large batches) or sixteen lanes per target.  A valid
//               upper bound T on r^2 of the (N_ngb+1)-th neighbour comes from
//               the target's Morton-order neighbours (64 on each side): their
//               (N_ngb+1)-th smallest r^2, bracketed in FP32 rounded up, so the
//               bound never falls below the exact value.  The wavefront then
//               walks the tree level by level against the box enclosing all its
//               targets' spheres (64 children tested per round, one coalesced
//               load), and each target's lanes keep the leaves that meet its
//               own sphere.
//
//  k_knn_bucket one wavefront per target.  The sub-buckets of its leaves that
//               meet the sphere, then their particles, two a lane a round; those
//               within the radius go to an LDS list, cut to the (N_ngb+1)-th
//               smallest when a round might not fit (bisection on ballot
//               counts); at the end each survivor's exact r^2 and its rank in
//               (r^2, ID, index) place it.
//
//  k_knn_team   the targets k_knn_bucket left (a leaf list that overflowed, a
//               group walk given up, a list that many equal r^2 kept from being
//               cut): a team of 16 lanes walks the tree from the root, nearest
//               child first, tests a leaf's 32 particles at once, cuts its list
//               by bisection on team-wide counts, and sorts it at the end
//               (register bitonic network; runs of equal r^2 placed by ID).
//
// Pruning is exact-conservative: a box gap is computed with the same rounded
// operations as a particle separation, and rounding is monotone, so no particle
// with r^2 <= the radius is ever skipped.  The result is the definition:
// the N_ngb smallest (r^2, id) among all other particles, in that order.
#include "sidm_internal.h"

namespace {

struct KnnArgs {
    int32_t *jsort;              // the rows in sorted indices too, [target in Morton order][k]
    const double *xs, *ys, *zs;
    const uint32_t *ids;
    const int32_t *perm;
    const double *nodes;
    const float4 *sbox;          // sub-bucket boxes: [2 s] lo, [2 s + 1] hi
    const int32_t *tlist, *slot;
    const int32_t *nt_dev;
    int32_t *ngb;
    double *h;
    unsigned int *derr;
    int32_t *list;       // [batch][SIDM_KNN_LMAX] leaf lists
    int32_t *nl;         // [batch] list length, -1 on overflow
    int32_t *fb_list;    // [batch] targets left to kernel B's root walk
    int32_t *fb_count;   // their number (cleared by the first kernel)
    double *tb;          // [batch] radius bound from the window
    TreeLevels lv;
    int64_t n, batch;
    int k;
    double box;
};

constexpr int32_t kIdxMask = (1 << SIDM_LEVEL_SHIFT) - 1;

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

// Upper bound on the K1-th smallest r^2, found by the LT lanes of a target:
// the K1-th smallest of the FP32 r^2 (rounded up) of the other particles
// within W places of the target in Morton order (W before and W after,
// shifted inward at the ends of the order).  Any K1 other particles bound the
// K1-th nearest from above, and rounding up keeps the bound valid.  The
// separations take no periodic image: a direct separation is never shorter
// than the nearest image's, so the bound stays valid, and Morton neighbours
// are direct neighbours except across a jump of the curve.  +inf if fewer
// than K1 values are finite.
template <bool PERIODIC, int LT, int W>
__device__ __forceinline__ double window_bound(const KnnArgs &A, int64_t i, double px, double py,
                                               double pz, int K1, int sub)
{
    constexpr int PER = (2 * W + 1 + LT - 1) / LT;
    const int64_t n = A.n;
    int64_t w0 = i - W;
    if (w0 > n - 1 - 2 * W) w0 = n - 1 - 2 * W;
    if (w0 < 0) w0 = 0;
    float v[PER];
    uint32_t lo = 0xffffffffu, hi = 0u;
    // positions requested three at a time (indices clamped into range, the
    // clamped results masked), then their separations
    constexpr int CH = 3;
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += CH) {
        double wx[CH], wy[CH], wz[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            int64_t j = w0 + (q0 + u) * LT + sub;
            if (j > n - 1) j = n - 1;
            if (q0 + u < PER) { wx[u] = A.xs[j]; wy[u] = A.ys[j]; wz[u] = A.zs[j]; }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int q = q0 + u;
            if (q >= PER) break;
            const int64_t j = w0 + q * LT + sub;
            v[q] = (j < n && j <= w0 + 2 * W && j != i)
                       ? __double2float_ru(sep2_sel<false>(px, py, pz, wx[u], wy[u], wz[u], A.box))
                       : INFINITY;
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (v[q] < INFINITY) {
            const uint32_t bv = __float_as_uint(v[q]);
            lo = bv < lo ? bv : lo;
            hi = bv > hi ? bv : hi;
        }
    }
    for (int off = 1; off < LT; off <<= 1) {
        const uint32_t ol = (uint32_t)__shfl_xor((int)lo, off);
        const uint32_t oh = (uint32_t)__shfl_xor((int)hi, off);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    auto count_le = [&](uint32_t bits) {
        const float f = __uint_as_float(bits);
        int c = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) c += v[q] <= f;
        for (int off = 1; off < LT; off <<= 1) c += __shfl_xor(c, off);
        return c;
    };
    if (lo > hi || count_le(hi) < K1) return INFINITY;
    // bisection on the FP32 bit patterns (monotone for values >= 0): the
    // smallest bracket end with >= K1 values at or below it; hi always has
    for (int it = 0; it < 14 && lo < hi; ++it) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (count_le(mid) >= K1) hi = mid; else lo = mid + 1;
    }
    return (double)__uint_as_float(hi);
}

// ---------------------------------------------------------------------------
// Kernel A: radius bound and per-target leaf list (a lane team per target)
// ---------------------------------------------------------------------------
constexpr int kFront = 512;               // frontier capacity of the level walk
constexpr int kLeafHits = 960;            // leaves a wavefront tests before its targets walk alone

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

// Level-synchronous walk of the tree for the lanes with member set, against
// the box enclosing their spheres: every round tests up to 64 children (one
// per lane, one coalesced load); surviving internal nodes form the next
// frontier, surviving leaves are offered to each member's own sphere (the LT
// lanes of a target take every LT-th leaf) and appended to its list; nl
// counts them all, also past the list's capacity.  Returns true if the walk
// gave up (frontier or leaf count too large), in which case the members'
// lists are incomplete.
template <bool PERIODIC, int LT>
__device__ __forceinline__ bool group_walk(const KnnArgs &A, int32_t (&s_fr)[2][kFront],
                                           double *s_hit, bool member, double px, double py,
                                           double pz, double T, double R, int32_t *lst, int &nl)
{
    const int lane = threadIdx.x;
    const double box = A.box;
    const double gxl = wave_min(member ? px - R : INFINITY), gxh = wave_max(member ? px + R : -INFINITY);
    const double gyl = wave_min(member ? py - R : INFINITY), gyh = wave_max(member ? py + R : -INFINITY);
    const double gzl = wave_min(member ? pz - R : INFINITY), gzh = wave_max(member ? pz + R : -INFINITY);
    // a group box inside the periodic box meets no image of a node, and the
    // members' spheres inside it meet no image of a leaf: then the walk tests
    // no images (the same decisions)
    const bool wrap = PERIODIC && !(gxl > 0.0 && gxh < box && gyl > 0.0 && gyh < box && gzl > 0.0 && gzh < box);
    int cur = 0, fn = 1, hits = 0;
    wave_sync();
    if (lane == 0) s_fr[0][0] = 0;                    // the root (top level, index 0)
    for (int lvl = A.lv.nlev - 1; lvl > 0; --lvl) {
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
                    hit = wrap ? (bx[0] <= bx[3] && interval_meets<true>(bx[0], bx[3], gxl, gxh, box) &&
                                  interval_meets<true>(bx[1], bx[4], gyl, gyh, box) &&
                                  interval_meets<true>(bx[2], bx[5], gzl, gzh, box))
                               : (bx[0] <= bx[3] && interval_meets<false>(bx[0], bx[3], gxl, gxh, box) &&
                                  interval_meets<false>(bx[1], bx[4], gyl, gyh, box) &&
                                  interval_meets<false>(bx[2], bx[5], gzl, gzh, box));
                }
            }
            const uint64_t m = __ballot(hit);
            const int rank = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            const int nh = __popcll(m);
            if (cl > 0) {
                if (nxt + nh > kFront) return true;
                if (hit) s_fr[cur ^ 1][nxt + rank] = (int32_t)q;
                nxt += nh;
            } else {
                hits += nh;
                if (hits > kLeafHits) return true;
                if (hit) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) s_hit[rank * 6 + d] = bx[d];
                    s_fr[cur ^ 1][rank] = (int32_t)q;
                }
                wave_sync();
                const int sub = lane % LT;
                const uint64_t mine = (LT == 64) ? ~0ull : ((1ull << LT) - 1ull);
                for (int h0 = 0; h0 < nh; h0 += LT) {
                    const int h = h0 + sub;
                    bool ok = false;
                    if (h < nh)
                        ok = member && (wrap ? box_gap2<true>(s_hit + h * 6, px, py, pz, box)
                                             : box_gap2<false>(s_hit + h * 6, px, py, pz, box)) <= T;
                    const uint64_t m = (__ballot(ok) >> (lane - sub)) & mine;
                    const int pos = nl + __popcll(m & ((1ull << sub) - 1ull));
                    if (ok && pos < SIDM_KNN_LMAX) lst[pos] = s_fr[cur ^ 1][h];
                    nl += __popcll(m);
                }
            }
        }
        cur ^= 1;
        fn = nxt;
    }
    return false;
}

template <bool PERIODIC, int LT>
__global__ __launch_bounds__(64) void k_knn_list(KnnArgs A, int64_t base, int64_t nblk)
{
    constexpr int G = 64 / LT;                // targets per wavefront
    __shared__ int32_t s_fr[2][kFront];
    __shared__ double s_hit[64 * 6];
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.fb_count = 0;
    const int64_t blk = xcd_block(nblk);
    if (blk < 0) return;
    const int nt = *A.nt_dev;
    const int lane = threadIdx.x, sub = lane % LT;
    const int64_t bb = blk * G + lane / LT;
    const int64_t b = base + bb;
    const bool valid = b < nt && bb < A.batch;
    if (!__any(valid)) return;
    const int32_t i = A.tlist[valid ? b : base + blk * G];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const double box = A.box;
    const double T = window_bound<PERIODIC, LT, 64>(A, i, px, py, pz, A.k + 1, sub);

    // sphere radius padded far beyond rounding, so a box a lane needs always
    // meets the group box
    const double R = sqrt(T) * (1.0 + 1e-9) + (fabs(px) + fabs(py) + fabs(pz) + box) * 1e-14;
    int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
    int nl = 0;
    // targets spread far apart (a jump of the Morton curve) would make the
    // group walk too long: then they walk the tree one by one in the second
    // kernel, as do targets with more than SIDM_KNN_LMAX leaves
    const bool gave_up = group_walk<PERIODIC, LT>(A, s_fr, s_hit, valid, px, py, pz, T, R, lst, nl);
    if (!valid || sub != 0) return;
    A.nl[bb] = (gave_up || nl > SIDM_KNN_LMAX) ? -1 : nl;
    A.tb[bb] = T;
}

// ---------------------------------------------------------------------------
// Kernel B: exact selection by a 16-lane team per target
// ---------------------------------------------------------------------------
constexpr int kStackB = 7 * 9 + 1;       // deepest walk: 10 levels (n < 2^31) of 8-ary nodes

// One compare-exchange stage (k = 2^LK, distance d = 2^LD) of an ascending
// bitonic sort on r^2 alone (payload jj) of TS*E keys held E per lane (lane tl
// of a team of TS lanes holds keys tl*E .. tl*E+E-1).  Equal keys are left in
// place, so no payload is duplicated.
template <int E, int LK, int LD>
__device__ __forceinline__ void rstage(double (&r)[E], int32_t (&jj)[E], int tl)
{
    constexpr int k = 1 << LK, d = 1 << LD;
    if constexpr (d < E) {
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const int bq = a ^ d;
            if (bq > a) {
                const bool up = (((tl * E + a) & k) == 0);
                const double ra = r[a], rb = r[bq];
                const bool sw = up ? (rb < ra) : (ra < rb);
                const int32_t ja = jj[a], jb = jj[bq];
                r[a] = sw ? rb : ra; r[bq] = sw ? ra : rb;
                jj[a] = sw ? jb : ja; jj[bq] = sw ? ja : jb;
            }
        }
    } else {
        constexpr int ld = d / E;
        const bool lower = (tl & ld) == 0;
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const double orr = __shfl_xor(r[a], ld);
            const int32_t oj = __shfl_xor(jj[a], ld);
            const bool up = (((tl * E + a) & k) == 0);
            const bool take = (lower == up) ? (orr < r[a]) : (r[a] < orr);
            r[a] = take ? orr : r[a];
            jj[a] = take ? oj : jj[a];
        }
    }
}

template <int E, int LK, int LD>
__device__ __forceinline__ void rmerge_steps(double (&r)[E], int32_t (&jj)[E], int tl)
{
    rstage<E, LK, LD>(r, jj, tl);
    if constexpr (LD > 0) rmerge_steps<E, LK, LD - 1>(r, jj, tl);
}

template <int E, int LK, int LOGN>
__device__ __forceinline__ void rlevels(double (&r)[E], int32_t (&jj)[E], int tl)
{
    rmerge_steps<E, LK, LK - 1>(r, jj, tl);
    if constexpr (LK < LOGN) rlevels<E, LK + 1, LOGN>(r, jj, tl);
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int E, int TS>
__device__ __forceinline__ void team_sort_r2(double (&r)[E], int32_t (&jj)[E], int tl)
{
    rlevels<E, 1, ilog2(TS * E)>(r, jj, tl);
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Next leaf of a root walk (targets whose list overflowed): pops the LDS
// stack, pushing the children within T nearest on top; -1 when empty.
template <bool PERIODIC, int TS>
__device__ __forceinline__ int32_t walk_next(const KnnArgs &A, int32_t *stk, int &sp, double T,
                                             double px, double py, double pz, int tl, int wteam)
{
    const double box = A.box;
    while (sp > 0) {
        --sp;
        const int32_t e = stk[sp];
        const int lvl = e >> SIDM_LEVEL_SHIFT;
        const int64_t q = e & kIdxMask;
        const double d2 = node_gap2<PERIODIC>(A.nodes, A.lv.off[lvl] + q, px, py, pz, box);
        if (!(d2 <= T)) continue;
        if (lvl == 0) return (int32_t)q;
        const int cl = lvl - 1;
        const int64_t cq = q * SIDM_TREE_FAN + tl;
        double gc = INFINITY;
        if (tl < SIDM_TREE_FAN && cq < A.lv.cnt[cl])
            gc = node_gap2<PERIODIC>(A.nodes, A.lv.off[cl] + cq, px, py, pz, box);
        const bool ok = gc <= T && gc < INFINITY;
        int rank = 0;
#pragma unroll
        for (int s2 = 0; s2 < SIDM_TREE_FAN; ++s2) {
            const double go = __shfl(gc, s2, TS);
            const bool oo = go <= T && go < INFINITY;
            rank += oo && (go < gc || (go == gc && s2 < tl));
        }
        const uint64_t m = (__ballot(ok) >> (wteam * TS)) & ((1ull << TS) - 1ull);
        const int np = __popcll(m);
        wave_sync();
        if (ok) stk[sp + np - 1 - rank] = (cl << SIDM_LEVEL_SHIFT) | (int32_t)cq;
        sp += np;
        wave_sync();
    }
    return -1;
}

// false: a step's leaves are tested as soon as their positions arrive, with no
// leaf of the next step in flight.  Requesting the next leaf ahead held more
// registers than the latency it hid was worth (measured slower at 10^6 and
// 256^3: the occupancy hides the latency instead)
constexpr bool kPrefetchLeaf = false;

// One target of kernel B (its team's lists and stack in LDS).
template <bool PERIODIC, int E, int TS, int LPI>
__device__ __forceinline__ void team_target(const KnnArgs &A, int64_t base, int64_t bb, double *L_r2,
                                            int32_t *L_j, int32_t *stk, int tl, int wteam)
{
    constexpr int N = TS * E;                 // list capacity
    constexpr int PPL = SIDM_LEAF / TS;       // particles of a leaf per lane
    constexpr int PS = PPL * LPI;             // particles per lane per step (LPI leaves)
    constexpr uint64_t TMASK = (TS == 64) ? ~0ull : ((1ull << TS) - 1ull);
    const int nt = *A.nt_dev;
    const int64_t b = base + bb;
    if (!(b < nt && bb < A.batch)) return;    // whole team
    const int32_t i = A.tlist[b];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const double box = A.box;
    const int64_t n = A.n;
    const int K1 = A.k + 1;
    const uint64_t below = (tl == 0) ? 0ull : ((1ull << tl) - 1ull);

    // a walk from the root, nearest child first (the targets come here when
    // their leaf list overflowed or kernel B' could not cut its list)
    int sp = 1;
    if (tl == 0) stk[0] = (A.lv.nlev - 1) << SIDM_LEVEL_SHIFT;
    double T = A.tb[bb];
    wave_sync();

    // leaf = 32 particles, PPL per lane (tl, tl + TS, ...); a step picks LPI
    // leaves, requests their positions and tests them (with kPrefetchLeaf the
    // next step's leaves are requested before the current ones are tested).
    // cur = -2 before the first leaf is picked, -1 once none is left.
    int32_t cur[LPI];
    double cx[PS], cy[PS], cz[PS];
#pragma unroll
    for (int u = 0; u < LPI; ++u) cur[u] = -2;
#pragma unroll
    for (int q = 0; q < PS; ++q) cx[q] = cy[q] = cz[q] = 0.0;
    int count = 0;
    bool finished = false;
    double r[E];
    int32_t jj[E];
    while (true) {
        int32_t nxt[LPI];
        double nx[PS], ny[PS], nz[PS];
#pragma unroll
        for (int u = 0; u < LPI; ++u) nxt[u] = -1;
#pragma unroll
        for (int q = 0; q < PS; ++q) nx[q] = ny[q] = nz[q] = 0.0;
        if (cur[0] != -1) {
#pragma unroll
            for (int u = 0; u < LPI; ++u) {
                if (u > 0 && nxt[u - 1] < 0) break;
                nxt[u] = walk_next<PERIODIC, TS>(A, stk, sp, T, px, py, pz, tl, wteam);
                if (nxt[u] >= 0) {
                    const int64_t s0 = (int64_t)nxt[u] * SIDM_LEAF;
#pragma unroll
                    for (int q = 0; q < PPL; ++q) {
                        const int64_t j = s0 + q * TS + tl < n ? s0 + q * TS + tl : s0;
                        const int qq = u * PPL + q;
                        nx[qq] = A.xs[j]; ny[qq] = A.ys[j]; nz[qq] = A.zs[j];
                    }
                }
            }
        }
        if constexpr (!kPrefetchLeaf) {
            // the picked leaves are tested in this step (their loads waited on)
#pragma unroll
            for (int u = 0; u < LPI; ++u) cur[u] = nxt[u];
#pragma unroll
            for (int q = 0; q < PS; ++q) { cx[q] = nx[q]; cy[q] = ny[q]; cz[q] = nz[q]; }
        }
#pragma unroll
        for (int u = 0; u < LPI; ++u) {
            if (cur[u] < 0) continue;
            const int64_t s0 = (int64_t)cur[u] * SIDM_LEAF;
            double rq[PPL];
            bool pq[PPL];
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const int qq = u * PPL + q;
                const int64_t j = s0 + q * TS + tl;
                rq[q] = sep2_sel<PERIODIC>(px, py, pz, cx[qq], cy[qq], cz[qq], box);
                pq[q] = j < n && rq[q] <= T && j != i;
            }
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const uint64_t m = (__ballot(pq[q]) >> (wteam * TS)) & TMASK;
                if (pq[q]) {
                    const int pos = count + __popcll(m & below);
                    L_r2[pos] = rq[q];
                    L_j[pos] = (int32_t)(s0 + q * TS + tl);
                }
                count += __popcll(m);
            }
        }
        // A team whose list might not hold the next step cuts it: the new
        // radius is the K1-th smallest r^2 rounded up to FP32, found by
        // bisection on team-wide counts (no sort), and entries above it are
        // dropped.  Teams that have run out of leaves wait; once all teams of
        // the wavefront have, they sort their lists together (exact FP64
        // r^2, equal values placed by ID) and keep the first K1.
        if (cur[0] == -1) finished = true;
        const bool need = !finished && count + LPI * SIDM_LEAF > N;
        const bool all_done = __all(finished);
        if (all_done || __any(need)) {
            wave_sync();
            if (all_done || need) {
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const int e = tl * E + q;
                    if (e < count) { jj[q] = L_j[e]; r[q] = L_r2[e]; }
                    else { r[q] = INFINITY; jj[q] = -1; }
                }
            }
            bool bad = false;
            if (need) {
                // the exact r^2 rounded up; the radius is the K1-th smallest
                // and an entry goes if its value exceeds it
                float f[E], fl[E];
                uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    f[q] = __double2float_ru(r[q]);
                    fl[q] = f[q];
                    if (tl * E + q < count) {
                        const uint32_t bv = __float_as_uint(f[q]);
                        lo = bv < lo ? bv : lo;
                        hi = bv > hi ? bv : hi;
                    }
                }
                for (int off = 1; off < TS; off <<= 1) {
                    const uint32_t ol = (uint32_t)__shfl_xor((int)lo, off);
                    const uint32_t oh = (uint32_t)__shfl_xor((int)hi, off);
                    lo = ol < lo ? ol : lo;
                    hi = oh > hi ? oh : hi;
                }
                // smallest bracket end with >= K1 values at or below it; stop
                // once few enough remain (the final sort orders the rest)
                int c_hi = count;
                for (int it = 0; it < 32 && lo < hi && c_hi > K1 + 8; ++it) {
                    const uint32_t mid = lo + ((hi - lo) >> 1);
                    const float fm = __uint_as_float(mid);
                    int c = 0;
#pragma unroll
                    for (int q = 0; q < E; ++q) c += f[q] <= fm;
                    for (int off = 1; off < TS; off <<= 1) c += __shfl_xor(c, off);
                    if (c >= K1) { hi = mid; c_hi = c; } else { lo = mid + 1; }
                }
                const float Tf = __uint_as_float(hi);
                // too many equal values to make room: sort and cut instead
                bad = c_hi > N - LPI * SIDM_LEAF;
                int mine = 0;
#pragma unroll
                for (int q = 0; q < E; ++q) mine += fl[q] <= Tf;
                int pre = mine;                        // inclusive prefix over the team
                for (int off = 1; off < TS; off <<= 1) {
                    const int o = __shfl_up(pre, off, TS);
                    if (tl >= off) pre += o;
                }
                int pos = pre - mine;
                wave_sync();
                if (!bad) {
#pragma unroll
                    for (int q = 0; q < E; ++q) {
                        if (fl[q] <= Tf) { L_r2[pos] = r[q]; L_j[pos] = jj[q]; ++pos; }
                    }
                    count = __shfl(pre, TS - 1, TS);
                    T = fmin(T, (double)Tf);
                }
            }
            const bool sort_now = all_done || (need && bad);
            if (sort_now) {
                team_sort_r2<E, TS>(r, jj, tl);
                // equal r^2 within the first K1 places: placed by ID below
                const double nx0 = __shfl(r[0], (tl + 1) % TS, TS);
                bool tie = false;
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const int e = tl * E + q;
                    const double nv = q + 1 < E ? r[q + 1] : nx0;
                    tie = tie || (e < K1 && e + 1 < count && e + 1 < N && r[q] == nv);
                }
                wave_sync();
                if ((__ballot(tie) >> (wteam * TS)) & TMASK) {
                    // rare (exact ties, e.g. on a lattice): place each element
                    // of a run of equal r^2 by its rank in (ID, index) in the run
#pragma unroll
                    for (int q = 0; q < E; ++q) { L_r2[tl * E + q] = r[q]; L_j[tl * E + q] = jj[q]; }
                    wave_sync();
                    int np[E];
                    for (int q = 0; q < E; ++q) {
                        const int e = tl * E + q;
                        np[q] = e;
                        if (!(r[q] < INFINITY)) continue;
                        int rs = e, re = e + 1;
                        while (rs > 0 && L_r2[rs - 1] == r[q]) --rs;
                        while (re < N && L_r2[re] == r[q]) ++re;
                        if (re - rs == 1) continue;
                        const uint32_t mid = A.ids[jj[q]];
                        int rank = rs;
                        for (int f = rs; f < re; ++f) {
                            const int32_t jf = L_j[f];
                            const uint32_t idf = A.ids[jf];
                            rank += (idf < mid) || (idf == mid && jf < jj[q]);
                        }
                        np[q] = rank;
                    }
                    wave_sync();
                    for (int q = 0; q < E; ++q)
                        if (np[q] < K1) { L_r2[np[q]] = r[q]; L_j[np[q]] = jj[q]; }
                } else {
#pragma unroll
                    for (int q = 0; q < E; ++q) {
                        const int e = tl * E + q;
                        if (e < K1) { L_r2[e] = r[q]; L_j[e] = jj[q]; }
                    }
                }
            }
            wave_sync();
            if (sort_now) {
                if (count >= K1) T = L_r2[K1 - 1];
                count = count < K1 ? count : K1;
            }
            if (all_done) break;
        }
#pragma unroll
        for (int u = 0; u < LPI; ++u) cur[u] = nxt[u];
#pragma unroll
        for (int q = 0; q < PS; ++q) { cx[q] = nx[q]; cy[q] = ny[q]; cz[q] = nz[q]; }
    }

    const int32_t a = A.slot[b];
    if (count < K1) {                          // cannot happen: T bounds K1 window particles
        if (tl == 0) atomicOr(A.derr, DERR_COUNT);
        return;
    }
    if (tl == 0) A.h[a] = sqrt(T);
    int32_t *out = A.ngb + (int64_t)a * A.k;
    int32_t *srt = A.jsort + b * A.k;
    for (int e = tl; e < A.k; e += TS) {
        const int32_t j = L_j[e];
        out[e] = A.perm[j];
        srt[e] = j;
    }
}

// Kernel B as the fallback of kernel B': a team per target of fb_list (the
// targets B' left), the grid striding over them.
template <bool PERIODIC, int E, int TS, int LPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_knn_team(KnnArgs A, int64_t base)
{
    constexpr int N = TS * E;
    constexpr int NT = 256 / TS;              // teams per workgroup
    __shared__ int32_t s_stack[NT][kStackB];  // only the overflow walk uses it
    __shared__ double s_r2[NT][N];
    __shared__ int32_t s_j[NT][N];
    const int team = threadIdx.x / TS, tl = threadIdx.x % TS;
    const int wteam = team % (64 / TS);       // team within the wavefront
    const int cnt = *A.fb_count;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t f0 = 0; f0 < cnt; f0 += stride) {
        const int64_t idx = f0 + (int64_t)blockIdx.x * NT + team;
        if (idx < cnt)
            team_target<PERIODIC, E, TS, LPI>(A, base, A.fb_list[idx], s_r2[team], s_j[team],
                                              s_stack[team], tl, wteam);
    }
}

// ---------------------------------------------------------------------------
// Kernel B': exact selection by one wavefront per target over sub-buckets
// ---------------------------------------------------------------------------
// The wavefront tests the sub-buckets of its target's leaf list (SIDM_SUB
// particles each, their own boxes; 128 a pass) against the radius and lists
// the kept ones in LDS.  Their particles are then tested kRound per lane a
// round (8 lanes a sub-bucket, all positions of a round requested together);
// those within the radius go to the target's LDS list as (r^2 rounded up to
// FP32, index) in one 64-bit word.  When a round might not fit, the list is
// cut: the radius becomes the K1-th smallest stored value, found by bisection
// on wavefront-wide counts (ballots), and larger entries go.  At the end the
// list is thinned the same way to at most 64 entries, each lane takes one,
// recomputes its exact r^2, and places it by its rank in (r^2, ID, index)
// among them.  Targets whose list overflowed in the first kernel, or whose
// list cannot be cut (many equal r^2), are left to kernel B's root walk.
constexpr int kSubPerLeaf = SIDM_LEAF / SIDM_SUB;
constexpr int kKeepMax = 384;                 // kept sub-buckets per target (more: the root walk)
constexpr int kRound = 2;                     // particles a lane tests per round (1, 3, 4 measured slower)
constexpr int kHitCap = 64 * (kRound + 2);    // list entries per target
constexpr int kHitQ = kHitCap / 64;           // list entries per lane
// dword 3 of a raw buffer resource on gfx9-family parts (32-bit data format)
constexpr int kRsrcWord3 = 0x00020000;

template <bool PERIODIC>
__device__ __forceinline__ double sub_gap2(const float4 &lo, const float4 &hi, double px, double py,
                                           double pz, double box)
{
    const double gx = axis_gap<PERIODIC>((double)lo.x, (double)hi.x, px, box);
    const double gy = axis_gap<PERIODIC>((double)lo.y, (double)hi.y, py, box);
    const double gz = axis_gap<PERIODIC>((double)lo.z, (double)hi.z, pz, box);
    const double g2 = (gx * gx + gy * gy) + gz * gz;
    return lo.x <= hi.x ? g2 : INFINITY;
}

// positions by 32-bit byte offsets into buffer resources (one address for the
// three loads), for arrays under 4 GiB
struct PosRsrc {
    __amdgpu_buffer_rsrc_t x, y, z;
};
__device__ __forceinline__ double buf_ld64(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <bool BUF>
__device__ __forceinline__ void load_pos(const KnnArgs &A, const PosRsrc &pr, int32_t j, double &x,
                                         double &y, double &z)
{
    if constexpr (BUF) {
        const uint32_t off = (uint32_t)j * 8u;
        x = buf_ld64(pr.x, off); y = buf_ld64(pr.y, off); z = buf_ld64(pr.z, off);
    } else {
        x = A.xs[j]; y = A.ys[j]; z = A.zs[j];
    }
}

// lanes below this one with their bit set in m
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
        v = o > v ? o : v;
    }
    return v;
}

// K1-th smallest of the FP32 bit patterns f (values >= 0, so the patterns
// order as the values) of the wavefront's entries q * 64 + lane < count: the
// smallest pattern with at least K1 entries at or below it, bisected until at
// most `enough` entries remain at or below it or the bracket closes.
// c_out = entries at or below the result.
template <int E>
__device__ __forceinline__ uint32_t wave_select(const uint32_t (&f)[E], int count, int K1, int enough,
                                                int &c_out)
{
    const int lane = threadIdx.x & 63;
    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if (q * 64 + lane < count) {
            lo = f[q] < lo ? f[q] : lo;
            hi = f[q] > hi ? f[q] : hi;
        }
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    int c_hi = count;
    for (int it = 0; it < 32 && lo < hi && c_hi > enough; ++it) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        int c = 0;
#pragma unroll
        for (int q = 0; q < E; ++q) c += __popcll(__ballot(q * 64 + lane < count && f[q] <= mid));
        if (c >= K1) { hi = mid; c_hi = c; } else { lo = mid + 1; }
    }
    c_out = c_hi;
    return hi;
}

// Keeps the entries whose pattern is at most Tf, in order, at the front of
// the list; returns their number.
template <int E>
__device__ __forceinline__ int wave_compact(uint64_t *L, double *R2, const uint32_t (&f)[E], uint32_t Tf,
                                            int count)
{
    const int lane = threadIdx.x & 63;
    uint64_t v[E];
    double r[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const bool in = q * 64 + lane < count;
        v[q] = in ? L[q * 64 + lane] : 0ull;
        r[q] = in ? R2[q * 64 + lane] : 0.0;
    }
    wave_sync();
    int total = 0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const bool keep = q * 64 + lane < count && f[q] <= Tf;
        const uint64_t m = __ballot(keep);
        if (keep) {
            L[total + lanes_below(m)] = v[q];
            R2[total + lanes_below(m)] = r[q];
        }
        total += __popcll(m);
    }
    wave_sync();
    return total;
}

__device__ __forceinline__ uint64_t hit_word(double r2, int32_t j)
{
    return ((uint64_t)__float_as_uint(__double2float_ru(r2)) << 32) | (uint32_t)j;
}

// The scan: returns false if the target must be left to the root walk.
// PER: with periodic images; a target whose padded sphere lies inside the box
// scans without them (no image of a particle within its radius can be nearer,
// and the separations of those within it round the same: bit-identical).
template <bool PER, bool BUF>
__device__ __forceinline__ bool wave_scan(const KnnArgs &A, const PosRsrc &pr, int32_t i, double px,
                                          double py, double pz, const int32_t *lst, int nl, uint32_t *K,
                                          uint64_t *L, double *R2, double &T, int &count)
{
    const int lane = threadIdx.x & 63;
    const double box = A.box;
    const int64_t n = A.n;
    const int K1 = A.k + 1;
    // 1. the kept sub-buckets
    int nk = 0;
    const int nsb = nl * kSubPerLeaf;
    for (int s0 = 0; s0 < nsb; s0 += 128) {
        int32_t sbi[2];
        float4 blo[2], bhi[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = s0 + u * 64 + lane;
            const int32_t leaf = t < nsb ? lst[t / kSubPerLeaf] : -1;
            sbi[u] = leaf >= 0 ? leaf * kSubPerLeaf + t % kSubPerLeaf : -1;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t q = sbi[u] >= 0 ? sbi[u] : 0;
            blo[u] = A.sbox[2 * q];
            bhi[u] = A.sbox[2 * q + 1];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const bool keep = sbi[u] >= 0 && sub_gap2<PER>(blo[u], bhi[u], px, py, pz, box) <= T;
            const uint64_t m = __ballot(keep);
            const int pos = nk + lanes_below(m);
            if (keep && pos < kKeepMax) K[pos] = (uint32_t)sbi[u];
            nk += __popcll(m);
        }
    }
    if (nk > kKeepMax) return false;
    wave_sync();
    // 2. their particles, kRound per lane a round
    for (int k0 = 0; k0 < nk; k0 += 8 * kRound) {
        double qx[kRound], qy[kRound], qz[kRound];
        int32_t jv[kRound];
        bool ok[kRound];
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const int e = k0 + u * 8 + (lane >> 3);
            const int32_t j = e < nk ? (int32_t)K[e] * SIDM_SUB + (lane & 7) : -1;
            ok[u] = j >= 0 && j < n && j != i;
            jv[u] = j;
            load_pos<BUF>(A, pr, ok[u] ? j : i, qx[u], qy[u], qz[u]);
        }
        double r2[kRound];
        bool hit[kRound];
        int nh = 0;
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            r2[u] = sep2_sel<PER>(px, py, pz, qx[u], qy[u], qz[u], box);
            hit[u] = ok[u] && r2[u] <= T;
            nh += __popcll(__ballot(hit[u]));
        }
        if (count + nh > kHitCap) {
            // cut: the radius becomes the K1-th smallest stored value
            uint32_t f[kHitQ];
#pragma unroll
            for (int q = 0; q < kHitQ; ++q)
                f[q] = q * 64 + lane < count ? (uint32_t)(L[q * 64 + lane] >> 32) : 0xffffffffu;
            int c_hi;
            const uint32_t Tf = wave_select<kHitQ>(f, count, K1, K1 + 8, c_hi);
            if (c_hi > kHitCap - 64 * kRound) return false;   // too many equal values
            count = wave_compact<kHitQ>(L, R2, f, Tf, count);
            T = fmin(T, (double)__uint_as_float(Tf));
#pragma unroll
            for (int u = 0; u < kRound; ++u) hit[u] = ok[u] && r2[u] <= T;
        }
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const uint64_t m = __ballot(hit[u]);
            if (hit[u]) {
                L[count + lanes_below(m)] = hit_word(r2[u], jv[u]);
                R2[count + lanes_below(m)] = r2[u];
            }
            count += __popcll(m);
        }
    }
    return true;
}

// Each lane's entries (RQ each, entry q * 64 + lane < count) placed by rank in
// (exact r^2, ID, index): rank < k to row place rank, rank k gives h.  The
// exact r^2 are those the scan stored beside the list.
template <int RQ>
__device__ __forceinline__ void wave_rank_out(const KnnArgs &A, const uint64_t *L, const double *R2,
                                              uint32_t *S, int count, int32_t *out, int32_t *srt,
                                              int32_t a)
{
    const int lane = threadIdx.x & 63;
    double re[RQ];
    int32_t je[RQ];
    int rank[RQ];
    wave_sync();
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int e = q * 64 + lane;
        je[q] = e < count ? (int32_t)(uint32_t)L[e] : -1;
        re[q] = e < count ? R2[e] : INFINITY;
        rank[q] = 0;
    }
    for (int f2 = 0; f2 < count; ++f2) {
        const double rf = R2[f2];
#pragma unroll
        for (int q = 0; q < RQ; ++q) rank[q] += rf < re[q];
    }
    // equal r^2 share a rank: each entry claims place rank, and a place
    // claimed twice shows a tie
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (je[q] >= 0) S[rank[q]] = (uint32_t)(q * 64 + lane);
    wave_sync();
    bool tie = false;
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (je[q] >= 0) tie = tie || S[rank[q]] != (uint32_t)(q * 64 + lane);
    wave_sync();
    if (__any(tie)) {
        uint32_t ide[RQ];
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            ide[q] = je[q] >= 0 ? A.ids[je[q]] : 0u;
            if (je[q] >= 0) S[q * 64 + lane] = ide[q];
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            if (je[q] < 0) continue;
            const int e = q * 64 + lane;
            for (int f2 = 0; f2 < count; ++f2) {
                if (R2[f2] != re[q] || f2 == e) continue;
                const uint32_t idf = S[f2];
                const int32_t jf = (int32_t)(uint32_t)L[f2];
                rank[q] += idf < ide[q] || (idf == ide[q] && jf < je[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        if (je[q] < 0) continue;
        if (rank[q] < A.k) {
            out[rank[q]] = A.perm[je[q]];
            srt[rank[q]] = je[q];
        } else if (rank[q] == A.k) {
            A.h[a] = sqrt(re[q]);
        }
    }
}

template <bool PERIODIC, bool BUF>
__device__ __forceinline__ void wave_target(const KnnArgs &A, int64_t base, int64_t bb, uint32_t *K,
                                            uint64_t *L, double *R2)
{
    const int lane = threadIdx.x & 63;
    const int nt = *A.nt_dev;
    const int64_t b = base + bb;
    if (!(b < nt && bb < A.batch)) return;
    const int nl = A.nl[bb];
    if (nl < 0) {                             // kernel B walks from the root
        if (lane == 0) A.fb_list[atomicAdd(A.fb_count, 1)] = (int32_t)bb;
        return;
    }
    const int32_t i = A.tlist[b];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const double box = A.box;
    const int64_t n = A.n;
    PosRsrc pr;
    const int nbytes = BUF ? (int)(uint32_t)(n * 8) : 0;
    pr.x = __builtin_amdgcn_make_buffer_rsrc((void *)A.xs, (short)0, nbytes, kRsrcWord3);
    pr.y = __builtin_amdgcn_make_buffer_rsrc((void *)A.ys, (short)0, nbytes, kRsrcWord3);
    pr.z = __builtin_amdgcn_make_buffer_rsrc((void *)A.zs, (short)0, nbytes, kRsrcWord3);
    const int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
    double T = A.tb[bb];
    int count = 0;
    // padded like the first kernel's sphere: far beyond rounding
    const double R = sqrt(T) * (1.0 + 1e-9) + (fabs(px) + fabs(py) + fabs(pz) + box) * 1e-14;
    const bool inside = px - R > 0.0 && px + R < box && py - R > 0.0 && py + R < box && pz - R > 0.0 &&
                        pz + R < box;
    const bool per = PERIODIC && !inside;
    const bool done = per ? wave_scan<PERIODIC, BUF>(A, pr, i, px, py, pz, lst, nl, K, L, R2, T, count)
                          : wave_scan<false, BUF>(A, pr, i, px, py, pz, lst, nl, K, L, R2, T, count);
    if (!done) {
        if (lane == 0) {
            A.nl[bb] = -1;
            A.fb_list[atomicAdd(A.fb_count, 1)] = (int32_t)bb;
        }
        return;
    }
    const int32_t a = A.slot[b];
    const int K1 = A.k + 1;
    if (count < K1) {                          // cannot happen: T bounds K1 window particles
        if (lane == 0) atomicOr(A.derr, DERR_COUNT);
        return;
    }
    wave_sync();
    if (count > 64) {
        uint32_t f[kHitQ];
#pragma unroll
        for (int q = 0; q < kHitQ; ++q)
            f[q] = q * 64 + lane < count ? (uint32_t)(L[q * 64 + lane] >> 32) : 0xffffffffu;
        int c_hi;
        const uint32_t Tf = wave_select<kHitQ>(f, count, K1, 64, c_hi);
        count = wave_compact<kHitQ>(L, R2, f, Tf, count);
    }
    int32_t *out = A.ngb + (int64_t)a * A.k;
    int32_t *srt = A.jsort + b * A.k;
    uint32_t *S = K;                           // the kept list is done with
    if (count <= 64) wave_rank_out<1>(A, L, R2, S, count, out, srt, a);
    else wave_rank_out<kHitQ>(A, L, R2, S, count, out, srt, a);
}

template <bool PERIODIC>
__global__ __launch_bounds__(256) void k_knn_bucket(KnnArgs A, int64_t base, int64_t nblk)
{
    constexpr int NW = 4;                     // wavefronts (targets) per workgroup
    static_assert(kKeepMax >= kHitCap, "the kept list's space holds the rank places");
    __shared__ uint32_t s_keep[NW][kKeepMax];
    __shared__ uint64_t s_hit[NW][kHitCap];
    __shared__ double s_r2[NW][kHitCap];
    const int w = threadIdx.x >> 6;
    const int64_t blk = xcd_block(nblk);
    if (blk < 0) return;
    const int64_t bb = blk * NW + w;
    if ((uint64_t)A.n * 8u <= 0xffffffffull)
        wave_target<PERIODIC, true>(A, base, bb, s_keep[w], s_hit[w], s_r2[w]);
    else
        wave_target<PERIODIC, false>(A, base, bb, s_keep[w], s_hit[w], s_r2[w]);
}

constexpr int kTeam = 16;                 // lanes per target in the team kernel (8 measured slower)

constexpr int kFallbackGrid = 2048;       // workgroups of the fallback launch (they stride over its targets)
constexpr int kLeavesPerStep = 2;          // leaves a team tests per step of its loop
// lanes per target in the leaf-list kernel: four (sixteen targets share a
// wavefront's group walk) for batches of at least kListWide targets, else
// sixteen (four targets a wavefront, more wavefronts for small batches).
// Measured: 256^3 box 78.5 -> 73.3 ms with four (8: 74.1); the 10^6 halo's
// 95,360 targets 0.49 ms with sixteen against 0.72 with four
constexpr int kListLanesWide = 4;
constexpr int kListLanesNarrow = 16;
constexpr int64_t kListWide = 1 << 18;

// per batch: leaf lists and bounds, the sub-bucket search, then the root
// walk (teams of TS lanes, lists of TS * E entries, LPI leaves a step) of the
// targets it left.  With several batches the root walk of a batch runs on the
// context's second stream while the next batch is searched: the batches
// alternate between two sets of counts, bounds and fallback lists (the leaf
// lists, which the walk does not read, are shared), and a set is reused only
// after the walk that read it has finished; the main stream waits for the
// last walks before the call returns.
template <bool P, int E, int TS>
hipError_t launch_batches(sidm_ctx *c, const KnnArgs &A0, int64_t n_active)
{
    hipError_t err = hipSuccess;
    auto keep = [&](hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; };
    // two leaves a step where the list leaves room for them after a cut
    constexpr int LPI = (TS * E >= 2 * SIDM_LEAF + 48) ? kLeavesPerStep : 1;
    const int64_t nb_cap = c->knn_batch;
    const hipStream_t s = c->stream;
    const bool fork = n_active > nb_cap;
    int t = 0;
    for (int64_t base = 0; base < n_active; base += nb_cap, ++t) {
        const int q = t & 1;
        KnnArgs A = A0;
        A.batch = (n_active - base) < nb_cap ? (n_active - base) : nb_cap;
        A.nl = c->knn_nl[q]; A.tb = c->knn_tb[q];
        A.fb_list = c->knn_fb[q]; A.fb_count = c->knn_fbn[q];
        if (fork && t >= 2) keep(hipStreamWaitEvent(s, c->knn_ev[q][1], 0));
        const int64_t gw = (A.batch + 3) / 4;
        if (A.batch >= kListWide) {
            constexpr int G = 64 / kListLanesWide;
            const int64_t gl = (A.batch + G - 1) / G;
            k_knn_list<P, kListLanesWide><<<xcd_grid(gl), 64, 0, s>>>(A, base, gl);
        } else {
            constexpr int G = 64 / kListLanesNarrow;
            const int64_t gl = (A.batch + G - 1) / G;
            k_knn_list<P, kListLanesNarrow><<<xcd_grid(gl), 64, 0, s>>>(A, base, gl);
        }
        k_knn_bucket<P><<<xcd_grid(gw), 256, 0, s>>>(A, base, gw);
        if (fork) {
            keep(hipEventRecord(c->knn_ev[q][0], s));
            keep(hipStreamWaitEvent(c->knn_aux, c->knn_ev[q][0], 0));
            k_knn_team<P, E, TS, LPI><<<kFallbackGrid, 256, 0, c->knn_aux>>>(A, base);
            keep(hipEventRecord(c->knn_ev[q][1], c->knn_aux));
        } else {
            k_knn_team<P, E, TS, LPI><<<kFallbackGrid, 256, 0, s>>>(A, base);
        }
    }
    if (fork) {
        keep(hipStreamWaitEvent(s, c->knn_ev[0][1], 0));
        if (t > 1) keep(hipStreamWaitEvent(s, c->knn_ev[1][1], 0));
    }
    return err;
}

}  // namespace

hipError_t launch_knn(sidm_ctx *c, int64_t n_active, int32_t *ngb, double *h)
{
    KnnArgs A;
    A.xs = c->xs; A.ys = c->ys; A.zs = c->zs;
    A.ids = c->ids; A.perm = c->perm; A.nodes = c->nodes;
    A.sbox = (const float4 *)c->sbox;
    A.tlist = c->tlist; A.slot = c->slot; A.nt_dev = c->nt_dev;
    A.ngb = ngb; A.h = h; A.derr = c->derr;
    A.jsort = c->jsort;
    A.list = c->knn_list;
    A.lv = c->lv;
    A.n = c->n; A.k = c->cfg.n_ngb; A.box = c->cfg.box; A.batch = 0;
    const bool per = c->cfg.periodic != 0;
    const bool small = A.k + 1 + 32 <= 64;       // list of 64 suffices for k <= 31
    phase_begin(c, PH_KNN);
    // both precision forms: the search is exact, so it is the FP64 one
    const int sel = (per ? 2 : 0) | (small ? 1 : 0);
    constexpr int B = 128 / kTeam, S = 64 / kTeam;   // lists of 128 and 64 entries
    hipError_t e;
    switch (sel) {
    case 0: e = launch_batches<false, B, kTeam>(c, A, n_active); break;
    case 1: e = launch_batches<false, S, kTeam>(c, A, n_active); break;
    case 2: e = launch_batches<true, B, kTeam>(c, A, n_active); break;
    default: e = launch_batches<true, S, kTeam>(c, A, n_active); break;
    }
    phase_end(c, PH_KNN);
    const hipError_t l = hipGetLastError();
    return e != hipSuccess ? e : l;
}
