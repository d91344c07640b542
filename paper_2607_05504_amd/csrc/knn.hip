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
//              exact value.  Each lane then walks the tree on its own (every
//              visit tests all children of a node at once, nearest first) and
//              records every leaf whose box lies within T, nearest first.
//
//  k_knn_team  a team of 16 lanes per target, four targets per wavefront.  The
//              team walks its leaf list, re-testing each leaf against the
//              current radius; a leaf's particles are loaded 16 at a time
//              (coalesced) and those within the radius are appended to a short
//              LDS list.  When the list fills it is sorted (register bitonic
//              network, 4 keys per lane) and cut back to N_ngb+1, which
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

template <bool PERIODIC, int W>
__global__ __launch_bounds__(64) void k_knn_list(KnnArgs A, int64_t base)
{
    __shared__ int32_t s_st[kStackA * 64];
    const int nt = *A.nt_dev;
    const int lane = threadIdx.x;
    const int64_t bb = (int64_t)blockIdx.x * 64 + lane;
    const int64_t b = base + bb;
    const bool valid = b < nt && bb < A.batch;
    if (!valid) return;
    const int32_t i = A.tlist[b];
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

    // per-lane walk: each visit tests all children of a node, nearest first
    int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
    int nl = 0;
    bool ovf = false;
    int sp = 1;
    s_st[lane] = (A.lv.nlev - 1) << SIDM_LEVEL_SHIFT;   // the root
    while (sp > 0 && !ovf) {
        --sp;
        const int32_t e = s_st[sp * 64 + lane];
        const int cl = (e >> SIDM_LEVEL_SHIFT) - 1;      // level of the children
        const int64_t q0 = (int64_t)(e & kIdxMask) * SIDM_TREE_FAN;
        const int64_t ccnt = A.lv.cnt[cl], coff = A.lv.off[cl];
        double g[SIDM_TREE_FAN];
        int32_t id[SIDM_TREE_FAN];
#pragma unroll
        for (int c = 0; c < SIDM_TREE_FAN; ++c) {
            const int64_t q = q0 + c;
            id[c] = (int32_t)q;
            g[c] = q < ccnt ? node_gap2<PERIODIC>(A.nodes, coff + q, px, py, pz, box) : INFINITY;
        }
        sort8(g, id);
        if (cl == 0) {
#pragma unroll
            for (int c = 0; c < SIDM_TREE_FAN; ++c) {
                if (g[c] <= T && g[c] < INFINITY) {
                    if (nl < SIDM_KNN_LMAX) lst[nl++] = id[c];
                    else ovf = true;
                }
            }
        } else {
#pragma unroll
            for (int c = SIDM_TREE_FAN - 1; c >= 0; --c) {
                if (g[c] <= T && g[c] < INFINITY) {
                    s_st[sp * 64 + lane] = (cl << SIDM_LEVEL_SHIFT) | id[c];
                    ++sp;
                }
            }
        }
    }
    A.nl[bb] = ovf ? -1 : nl;
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

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

template <bool PERIODIC, int E>
__global__ __launch_bounds__(256) void k_knn_team(KnnArgs A, int64_t base)
{
    constexpr int N = 16 * E;                 // list capacity
    constexpr int SCAP = SIDM_KNN_LMAX + kStackA;
    __shared__ int32_t s_stack[16][SCAP];
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

    // work stack: the leaf list (nearest on top), or the root on overflow.
    // Entries are packed (level << SIDM_LEVEL_SHIFT) | index; leaves are level 0.
    const int nl = A.nl[bb];
    int sp;
    if (nl >= 0) {
        const int32_t *lst = A.list + bb * SIDM_KNN_LMAX;
        for (int t = tl; t < nl; t += 16) stk[nl - 1 - t] = lst[t];
        sp = nl;
    } else {
        if (tl == 0) stk[0] = (A.lv.nlev - 1) << SIDM_LEVEL_SHIFT;
        sp = 1;
    }
    wave_sync();

    double T = A.tb[bb];
    int count = 0;
    double r[E];
    uint32_t id[E];
    int32_t jj[E];
    const uint64_t below = (tl == 0) ? 0ull : ((1ull << tl) - 1ull);
    int64_t cur_s0 = 0;
    int cur_m = 0, cur_off = 0;
    bool done = false;
    while (true) {
        if (done || count + 16 > N) {
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
            if (done) break;
        }
        if (cur_off >= cur_m) {
            // next leaf within the radius
            cur_m = 0;
            cur_off = 0;
            while (sp > 0) {
                --sp;
                const int32_t e = stk[sp];
                const int lvl = e >> SIDM_LEVEL_SHIFT;
                const int64_t q = e & kIdxMask;
                const double d2 = node_gap2<PERIODIC>(A.nodes, A.lv.off[lvl] + q, px, py, pz, box);
                if (!(d2 <= T)) continue;
                if (lvl == 0) {
                    cur_s0 = q * SIDM_LEAF;
                    cur_m = (int)((n - cur_s0) < SIDM_LEAF ? (n - cur_s0) : SIDM_LEAF);
                    break;
                }
                // overflow path: push the children within the radius
                const int cl = lvl - 1;
                const int64_t cq = q * SIDM_TREE_FAN + tl;
                double gc = INFINITY;
                if (tl < SIDM_TREE_FAN && cq < A.lv.cnt[cl])
                    gc = node_gap2<PERIODIC>(A.nodes, A.lv.off[cl] + cq, px, py, pz, box);
                const bool ok = gc <= T && gc < INFINITY;
                // rank among the passing children by (gap, index); nearest on top
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
            }
            if (cur_m == 0) { done = true; continue; }
        }
        // 16 particles of the current leaf
        const int c = cur_off + tl;
        const int64_t j = cur_s0 + c;
        bool pass = false;
        double r2 = 0.0;
        if (c < cur_m) {
            r2 = sep2_sel<PERIODIC>(px, py, pz, A.xs[j], A.ys[j], A.zs[j], box);
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
