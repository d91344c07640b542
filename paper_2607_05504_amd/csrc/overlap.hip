// Kernel-overlap estimator (sec. 4.2, Eq. kernelOverlap, and the paper's
// appendix on the overlap kernel): the geometric factor of a pair is the
// overlap integral of the two particles' cubic splines, so the partners of i
// are all j with r_ij < h_i + h_j and the search needs every particle's h.
//
//  k_overlap_table  ghat(alpha, rho) at the table nodes, one thread each: the
//                   overlap of splines with h_i = alpha, h_j = 1 - alpha at
//                   separation rho.  For two radial kernels, in spherical
//                   coordinates about x_i (s = |x - x_i|, t = |x - x_j|),
//                     g(r) = 2 pi / r  int s W_i(s) [F_j(r + s) - F_j(|r - s|)] ds
//                   with F_j(t) = int_0^t t' W_j(t') dt' in closed form; the
//                   outer integrand is a polynomial of degree <= 9 between
//                   breakpoints, so a 5-point Gauss-Legendre rule per piece is
//                   exact.  alpha = 0 is a point partner: ghat = W(rho, 1).
//  k_update_h       (optional) the active particles' new h into h_all
//  k_gather_h       every particle's h into Morton order (each checked > 0 and
//                   finite), then k_leaf_hmax / k_level_hmax: the largest h
//                   below every node of the tree, level after level (the
//                   tree update between the two walks the paper describes)
//  k_overlap        a team of 8 lanes per active particle walks the tree from
//                   the root (one node per step, its 8 children tested by the
//                   8 lanes), opening a child whose box lies closer than
//                   h_i + h_max(child), and tests a leaf's 32 particles four
//                   per lane, appending each j with r_ij^2 < (h_i + h_j)^2 to
//                   the target's row.
//
// The pruning is conservative under rounding: a box gap rounds like a
// particle separation (never above it) and h_i + h_j <= h_i + h_max rounds
// monotonically, so no partner is skipped; the result is the definition.
#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kTeamO = SIDM_TREE_FAN;      // lanes per target: one per child of a node
constexpr int kStackO = (SIDM_TREE_FAN - 1) * (SIDM_MAX_LEVELS - 1) + 1;   // depth-first bound

// F(x) = int_0^x q w(q) dq for the unit-support spline w(q) = W(q, 1)
__device__ double spline_moment(double x)
{
    const double c = 8.0 / SIDM_PI;
    if (x <= 0.5) {
        const double x2 = x * x;
        return c * ((0.5 * x2 - 1.5 * (x2 * x2)) + 1.2 * ((x2 * x2) * x));
    }
    // antiderivative of q (1 - q)^3: -q (1 - q)^4 / 4 - (1 - q)^5 / 20
    auto A = [](double q) {
        const double u = 1.0 - q, u4 = (u * u) * (u * u);
        return -0.25 * q * u4 - 0.05 * (u4 * u);
    };
    const double half = c * ((0.5 * 0.25 - 1.5 * 0.0625) + 1.2 * 0.03125);
    const double xe = x < 1.0 ? x : 1.0;
    return half + 2.0 * c * (A(xe) - A(0.5));
}

// 5-point Gauss-Legendre rule on [-1, 1]
struct GL5 { double x[5], w[5]; };

__device__ GL5 gl5()
{
    GL5 g;
    const double a = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
    const double b = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
    const double wa = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
    const double wb = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
    g.x[0] = -b; g.x[1] = -a; g.x[2] = 0.0; g.x[3] = a; g.x[4] = b;
    g.w[0] = wb; g.w[1] = wa; g.w[2] = 128.0 / 225.0; g.w[3] = wa; g.w[4] = wb;
    return g;
}

// the exact overlap of splines with supports hi and hj at separation r
__device__ double overlap_exact(double hi, double hj, double r)
{
    if (!(r < hi + hj)) return 0.0;
    const GL5 g = gl5();
    double cut[10];
    int nc = 0;
    if (r == 0.0) {
        // 4 pi int s^2 W_i(s) W_j(s) ds up to the smaller support
        const double top = hi < hj ? hi : hj;
        const double cand[4] = {0.0, 0.5 * hi, 0.5 * hj, top};
        for (int c = 0; c < 4; ++c)
            if (cand[c] <= top) cut[nc++] = cand[c];
    } else {
        const double cand[10] = {0.0, hi, 0.5 * hi, r, r - 0.5 * hj, r + 0.5 * hj,
                                 r - hj, r + hj, 0.5 * hj - r, hj - r};
        for (int c = 0; c < 10; ++c)
            if (cand[c] >= 0.0 && cand[c] <= hi) cut[nc++] = cand[c];
    }
    for (int p = 1; p < nc; ++p) {           // insertion sort of the breakpoints
        const double t = cut[p];
        int q = p - 1;
        while (q >= 0 && cut[q] > t) { cut[q + 1] = cut[q]; --q; }
        cut[q + 1] = t;
    }
    double sum = 0.0;
    for (int p = 0; p + 1 < nc; ++p) {
        const double lo = cut[p], up = cut[p + 1];
        if (!(up > lo)) continue;
        const double mid = 0.5 * (lo + up), half = 0.5 * (up - lo);
        double part = 0.0;
        for (int q = 0; q < 5; ++q) {
            const double s = mid + half * g.x[q];
            double f;
            if (r == 0.0) {
                f = (s * s) * cubic_spline(s, hi) * cubic_spline(s, hj);
            } else {
                const double Fp = spline_moment((r + s) / hj), Fm = spline_moment(fabs(r - s) / hj);
                f = s * cubic_spline(s, hi) * ((Fp - Fm) / hj);
            }
            part += g.w[q] * f;
        }
        sum += half * part;
    }
    return r == 0.0 ? 4.0 * SIDM_PI * sum : (2.0 * SIDM_PI / r) * sum;
}

__global__ __launch_bounds__(kBlock) void k_overlap_table(double *tab)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    constexpr int NR1 = SIDM_OVERLAP_NR + 1;
    if (t >= (SIDM_OVERLAP_NA + 1) * NR1) return;
    const int a = t / NR1, b = t - a * NR1;
    const double al = (double)a / (2.0 * SIDM_OVERLAP_NA);
    const double rho = (double)b / SIDM_OVERLAP_NR;
    tab[t] = a == 0 ? cubic_spline(rho, 1.0) : overlap_exact(al, 1.0 - al, rho);
}

// the active particles' new smoothing lengths into every particle's h, through
// the active set's mapping (target b: Morton index tlist[b], slot slot[b])
__global__ __launch_bounds__(kBlock) void k_update_h(const int32_t *__restrict__ tlist,
                                                     const int32_t *__restrict__ slot,
                                                     const int32_t *__restrict__ nt_dev,
                                                     const int32_t *__restrict__ perm,
                                                     const double *__restrict__ h_active,
                                                     double *h_all)
{
    const int64_t nt = *nt_dev;
    for (int64_t b = blockIdx.x * (int64_t)kBlock + threadIdx.x; b < nt;
         b += (int64_t)gridDim.x * kBlock)
        h_all[perm[tlist[b]]] = h_active[slot[b]];
}

__global__ __launch_bounds__(kBlock) void k_gather_h(int64_t n, const int32_t *__restrict__ perm,
                                                     const double *__restrict__ h_all, double *hs,
                                                     unsigned int *derr)
{
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        double h = h_all[perm[t]];
        if (!(h > 0.0) || !(h < 1e300)) {
            atomicOr(derr, DERR_BAD_H);
            h = 0.0;
        }
        hs[t] = h;
    }
}

// largest h of each leaf: 32 lanes a leaf, butterfly max
__global__ __launch_bounds__(kBlock) void k_leaf_hmax(int64_t n, int64_t nleaf,
                                                      const double *__restrict__ hs, double *hmax)
{
    const int64_t leaf = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 5;
    const int sub = threadIdx.x & 31;
    const int64_t s = leaf * SIDM_LEAF + sub;
    double v = (leaf < nleaf && s < n) ? hs[s] : 0.0;
    for (int off = 16; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 32));
    if (sub == 0 && leaf < nleaf) hmax[leaf] = v;
}

__global__ __launch_bounds__(kBlock) void k_level_hmax(double *hmax, int64_t off_child,
                                                       int64_t cnt_child, int64_t off, int64_t cnt)
{
    const int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (q >= cnt) return;
    double v = 0.0;
    for (int c = 0; c < SIDM_TREE_FAN; ++c) {
        const int64_t ch = q * SIDM_TREE_FAN + c;
        if (ch >= cnt_child) break;
        v = fmax(v, hmax[off_child + ch]);
    }
    hmax[off + q] = v;
}

// LDS written by some lanes of a wavefront, read by others next
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct OvlArgs {
    const double *xs, *ys, *zs, *hs, *hmax, *nodes;
    const int32_t *perm, *tlist, *slot, *nt_dev;
    int32_t *ngb, *count;
    unsigned int *derr;
    TreeLevels lv;
    int64_t n;
    double box;
    int32_t max_ngb;
};

template <bool PERIODIC>
__global__ __launch_bounds__(kBlock) void k_overlap(OvlArgs A)
{
    __shared__ int32_t s_stk[kBlock / kTeamO][kStackO];
    const int team = threadIdx.x / kTeamO, tl = threadIdx.x % kTeamO;
    const int wteam = (threadIdx.x & 63) / kTeamO;
    const int64_t b = (int64_t)blockIdx.x * (kBlock / kTeamO) + team;
    if (b >= *A.nt_dev) return;                 // whole teams leave together
    int32_t *stk = s_stk[team];
    const int32_t i = A.tlist[b], a = A.slot[b];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i], hi = A.hs[i];
    const double box = A.box;
    const uint64_t below = (1ull << tl) - 1ull;
    int32_t *row = A.ngb + (int64_t)a * A.max_ngb;
    int64_t cnt = 0;
    const int top = A.lv.nlev - 1;
    if (tl == 0) stk[0] = top << SIDM_LEVEL_SHIFT;
    int sp = 1;
    wave_lds_sync();
    while (sp > 0) {
        const int32_t e = stk[--sp];
        const int lvl = e >> SIDM_LEVEL_SHIFT;
        const int64_t q = e & ((1 << SIDM_LEVEL_SHIFT) - 1);
        if (lvl == 0) {
            const int64_t j0 = q * SIDM_LEAF;
#pragma unroll
            for (int rep = 0; rep < SIDM_LEAF / kTeamO; ++rep) {
                const int64_t j = j0 + rep * kTeamO + tl;
                bool ok = false;
                if (j < A.n && j != i) {
                    const double r2 = sep2<PERIODIC>(px, py, pz, A.xs[j], A.ys[j], A.zs[j], box);
                    const double s = hi + A.hs[j];
                    ok = r2 < s * s;
                }
                const uint64_t m = (__ballot(ok) >> (wteam * kTeamO)) & 0xffull;
                if (ok) {
                    const int64_t pos = cnt + __popcll(m & below);
                    if (pos < A.max_ngb) row[pos] = A.perm[j];
                }
                cnt += __popcll(m);
            }
            continue;
        }
        const int cl = lvl - 1;
        const int64_t cq = q * SIDM_TREE_FAN + tl;
        bool ok = false;
        if (cq < A.lv.cnt[cl]) {
            const int64_t g = A.lv.off[cl] + cq;
            const double R = hi + A.hmax[g];
            ok = node_gap2<PERIODIC>(A.nodes, g, px, py, pz, box) < R * R;
        }
        const uint64_t m = (__ballot(ok) >> (wteam * kTeamO)) & 0xffull;
        const int np = __popcll(m);
        wave_lds_sync();
        if (ok && sp + np <= kStackO) stk[sp + __popcll(m & below)] = (cl << SIDM_LEVEL_SHIFT) | (int32_t)cq;
        if (sp + np > kStackO) {                // cannot happen: depth-first bound
            if (tl == 0) atomicOr(A.derr, DERR_STALL);
            break;
        }
        sp += np;
        wave_lds_sync();
    }
    if (tl == 0) {
        A.count[a] = (int32_t)(cnt < 0x7fffffff ? cnt : 0x7fffffff);
        if (cnt > A.max_ngb) atomicOr(A.derr, DERR_NGB_OVERFLOW);
    }
}

int grid_for(int64_t n, int cap = 4096)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

}  // namespace

hipError_t launch_overlap_table(sidm_ctx *c)
{
    constexpr int nodes = (SIDM_OVERLAP_NA + 1) * (SIDM_OVERLAP_NR + 1);
    k_overlap_table<<<(nodes + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(c->gtab);
    return hipGetLastError();
}

hipError_t launch_find_overlap(sidm_ctx *c, double *h_all, const double *h_active,
                               int64_t n_active, int32_t max_ngb, int32_t *ngb, int32_t *count)
{
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    const TreeLevels &lv = c->lv;
    phase_begin(c, PH_OVERLAP);
    if (h_active)
        k_update_h<<<grid_for(n_active), kBlock, 0, s>>>(c->tlist, c->slot, c->nt_dev, c->perm,
                                                         h_active, h_all);
    k_gather_h<<<grid_for(n), kBlock, 0, s>>>(n, c->perm, h_all, c->hs, c->derr);
    const int64_t nleaf = lv.cnt[0];
    k_leaf_hmax<<<(unsigned)((nleaf * 32 + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, nleaf, c->hs,
                                                                                c->hmax);
    for (int l = 1; l < lv.nlev; ++l)
        k_level_hmax<<<(unsigned)((lv.cnt[l] + kBlock - 1) / kBlock), kBlock, 0, s>>>(
            c->hmax, lv.off[l - 1], lv.cnt[l - 1], lv.off[l], lv.cnt[l]);
    OvlArgs A;
    A.xs = c->xs; A.ys = c->ys; A.zs = c->zs; A.hs = c->hs; A.hmax = c->hmax; A.nodes = c->nodes;
    A.perm = c->perm; A.tlist = c->tlist; A.slot = c->slot; A.nt_dev = c->nt_dev;
    A.ngb = ngb; A.count = count; A.derr = c->derr;
    A.lv = lv; A.n = n; A.box = c->cfg.box; A.max_ngb = max_ngb;
    const unsigned grid = (unsigned)((n_active + kBlock / kTeamO - 1) / (kBlock / kTeamO));
    if (c->cfg.periodic) k_overlap<true><<<grid, kBlock, 0, s>>>(A);
    else k_overlap<false><<<grid, kBlock, 0, s>>>(A);
    phase_end(c, PH_OVERLAP);
    return hipGetLastError();
}
