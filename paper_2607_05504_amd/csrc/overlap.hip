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
//  k_overlap        one wavefront per group of 4 targets consecutive in Morton
//                   order.  The group walks the tree once against its bounding
//                   sphere (centre c, radius rg): a node is opened when its box
//                   lies closer to c than hg + h_max(node) + rg, hg the group's
//                   largest h, up to 8 nodes popped per step (64 lanes, one per
//                   child).  A leaf that passes gets the mask of the targets i
//                   whose own test, box closer than h_i + h_max(leaf), it
//                   passes, and is listed in LDS unless that mask is empty.
//                   The listed leaves are then read two at a time (32 lanes
//                   each), and each target in the pair's masks tests all 64
//                   particles, appending each j with r_ij^2 < (h_i + h_j)^2 to
//                   its row.  A leaf's particles are thus read once for the
//                   whole group.
//
// The pruning is conservative under rounding: a box gap rounds like a
// particle separation (never above it) and h_i + h_j <= h_i + h_max rounds
// monotonically, so the per-target leaf test skips no partner; the group test
// only widens it (by the margins given at its use).  The result is the
// definition.
#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kGroup = 4;                   // targets per wavefront in the walk
// The walk pops up to 8 nodes at a time from the top of a stack kept sorted
// by depth (children go above the rest, those of lower entries lower), so a
// level's nodes are pushed only once none of that level is left: at most
// 64 per level below the root.
constexpr int kStackG = 64 * (SIDM_MAX_LEVELS - 1);
constexpr int kLeafCap = 192;              // leaves listed per batch (a walk step adds <= 64)

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
    int64_t n, nblk;
    double box;
    int32_t max_ngb;
};

template <bool PERIODIC>
__global__ __launch_bounds__(kBlock) void k_overlap(OvlArgs A)
{
    __shared__ int32_t s_stk[kWaves][kStackG];
    __shared__ int32_t s_leaf[kWaves][kLeafCap];
    __shared__ int32_t s_lmsk[kWaves][kLeafCap];
    __shared__ double s_tgt[kWaves][kGroup][4];
    __shared__ int64_t s_off[SIDM_MAX_LEVELS], s_cnt[SIDM_MAX_LEVELS];
    if (threadIdx.x < SIDM_MAX_LEVELS) {
        s_off[threadIdx.x] = A.lv.off[threadIdx.x];
        s_cnt[threadIdx.x] = A.lv.cnt[threadIdx.x];
    }
    __syncthreads();
    const int64_t blk = xcd_block(A.nblk);
    if (blk < 0) return;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nt = *A.nt_dev;
    const int64_t b0 = (blk * kWaves + wv) * kGroup;
    if (b0 >= nt) return;                       // whole wavefronts leave together
    const int ng = nt - b0 < kGroup ? (int)(nt - b0) : kGroup;
    int32_t *stk = s_stk[wv], *lbuf = s_leaf[wv], *lmsk = s_lmsk[wv];
    double (*tgt)[4] = s_tgt[wv];
    const double box = A.box;
    const int64_t n = A.n;
    const uint64_t below = (1ull << lane) - 1ull;

    // the group's targets: Morton index, row, and (x, y, z, h) in LDS; the
    // padding slots of a short last group repeat its first target
    int32_t ti[kGroup], ta[kGroup], cnt[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        const int64_t b = b0 + (t < ng ? t : 0);
        ti[t] = A.tlist[b];
        ta[t] = A.slot[b];
        cnt[t] = 0;
    }
    double mx = 0.0, my = 0.0, mz = 0.0, mh = 0.0;  // lane t < kGroup: target t
    {
        int32_t it = ti[0];
#pragma unroll
        for (int t = 1; t < kGroup; ++t)
            if (lane == t) it = ti[t];
        if (lane < kGroup) {
            mx = A.xs[it]; my = A.ys[it]; mz = A.zs[it]; mh = A.hs[it];
            tgt[lane][0] = mx; tgt[lane][1] = my; tgt[lane][2] = mz; tgt[lane][3] = mh;
        }
    }
    // bounding sphere of the group (centre c, radius rg) and its largest h
    double lx = mx, ux = mx, ly = my, uy = my, lz = mz, uz = mz, hg = mh;
    if (lane >= kGroup) { lx = ly = lz = INFINITY; ux = uy = uz = -INFINITY; }
#pragma unroll
    for (int off = 1; off < kGroup; off <<= 1) {
        lx = fmin(lx, __shfl_xor(lx, off)); ux = fmax(ux, __shfl_xor(ux, off));
        ly = fmin(ly, __shfl_xor(ly, off)); uy = fmax(uy, __shfl_xor(uy, off));
        lz = fmin(lz, __shfl_xor(lz, off)); uz = fmax(uz, __shfl_xor(uz, off));
        hg = fmax(hg, __shfl_xor(hg, off));
    }
    const double cx = __shfl(0.5 * (lx + ux), 0), cy = __shfl(0.5 * (ly + uy), 0),
                 cz = __shfl(0.5 * (lz + uz), 0);
    double d2 = 0.0;
    if (lane < kGroup) {
        const double dx = mx - cx, dy = my - cy, dz = mz - cz;
        d2 = (dx * dx + dy * dy) + dz * dz;
    }
#pragma unroll
    for (int off = 1; off < kGroup; off <<= 1) d2 = fmax(d2, __shfl_xor(d2, off));
    // A node can hold a partner of some target only if its box lies closer to
    // c than hg + h_max(node) + rg (triangle inequality); the relative and, in
    // a periodic box, absolute margins of 2^-40 cover every rounding.
    constexpr double kRel = 1.0 + 0x1p-40;
    const double r0 = __shfl((hg + sqrt(d2)) * kRel + (PERIODIC ? box * 0x1p-40 : 0.0), 0);
    wave_lds_sync();

    int sp = 1, nl = 0;
    if (lane == 0) stk[0] = (A.lv.nlev - 1) << SIDM_LEVEL_SHIFT;
    wave_lds_sync();
    while (true) {
        // Walk until the stack is empty or the leaf list could overflow.  Pop
        // the top k <= 8 nodes; lane 8e + c tests child c of popped node e
        // (e = 0 the lowest in the stack).  An accepted leaf carries the mask
        // of the targets whose own test (gap < h_i + h_max(leaf)) it passes,
        // and is dropped when that mask is empty.
        while (sp > 0 && nl <= kLeafCap - 64) {
            const int k = sp < 8 ? sp : 8;
            const int e = lane >> 3, ch = lane & 7;
            bool okN = false, okL = false;
            int32_t ent = 0, tm = 0;
            if (e < k) {
                const int32_t pe = stk[sp - k + e];
                const int cl = (pe >> SIDM_LEVEL_SHIFT) - 1;
                const int64_t cq = (int64_t)(pe & ((1 << SIDM_LEVEL_SHIFT) - 1)) * SIDM_TREE_FAN + ch;
                if (cq < s_cnt[cl]) {
                    const int64_t g = s_off[cl] + cq;
                    const double *nb = A.nodes + g * 6;
                    const double bx0 = nb[0], by0 = nb[1], bz0 = nb[2];
                    const double bx1 = nb[3], by1 = nb[4], bz1 = nb[5];
                    const double hm = A.hmax[g];
                    if (bx0 <= bx1) {
                        const double gx = axis_gap<PERIODIC>(bx0, bx1, cx, box);
                        const double gy = axis_gap<PERIODIC>(by0, by1, cy, box);
                        const double gz = axis_gap<PERIODIC>(bz0, bz1, cz, box);
                        const double R = r0 + hm * kRel;
                        if ((gx * gx + gy * gy) + gz * gz < R * R) {
                            if (cl > 0) {
                                okN = true;
                                ent = (cl << SIDM_LEVEL_SHIFT) | (int32_t)cq;
                            } else {
#pragma unroll
                                for (int t = 0; t < kGroup; ++t) {
                                    const double *T = tgt[t];
                                    const double ex = axis_gap<PERIODIC>(bx0, bx1, T[0], box);
                                    const double ey = axis_gap<PERIODIC>(by0, by1, T[1], box);
                                    const double ez = axis_gap<PERIODIC>(bz0, bz1, T[2], box);
                                    const double Rt = T[3] + hm;
                                    if (t < ng && (ex * ex + ey * ey) + ez * ez < Rt * Rt)
                                        tm |= 1 << t;
                                }
                                okL = tm != 0;
                                ent = (int32_t)cq;
                            }
                        }
                    }
                }
            }
            const uint64_t mN = __ballot(okN), mL = __ballot(okL);
            const int base = sp - k, np = __popcll(mN);
            if (base + np > kStackG) {          // cannot happen: see kStackG
                if (lane == 0) atomicOr(A.derr, DERR_STALL);
                sp = 0;
                nl = 0;
                break;
            }
            wave_lds_sync();
            if (okN) stk[base + __popcll(mN & below)] = ent;
            if (okL) {
                const int at = nl + __popcll(mL & below);
                lbuf[at] = ent;
                lmsk[at] = tm;
            }
            sp = base + np;
            nl += __popcll(mL);
            wave_lds_sync();
        }
        // The listed leaves two at a time (lanes 0-31 one, 32-63 the other);
        // an odd leaf waits for the next batch unless the walk is done.
        const int avail = sp == 0 ? nl : (nl & ~1);
        const int half = lane >> 5, lt = lane & 31;
        for (int u = 0; u < avail; u += 2) {
            const int need = __builtin_amdgcn_readfirstlane(lmsk[u] | (u + 1 < avail ? lmsk[u + 1] : 0));
            const int32_t lf = u + half < avail ? lbuf[u + half] : -1;
            const int64_t j = (int64_t)lf * SIDM_LEAF + lt;
            const bool valid = lf >= 0 && j < n;
            double xj = 0.0, yj = 0.0, zj = 0.0, hj = 0.0;
            int32_t pj = 0;
            if (valid) { xj = A.xs[j]; yj = A.ys[j]; zj = A.zs[j]; hj = A.hs[j]; pj = A.perm[j]; }
#pragma unroll
            for (int t = 0; t < kGroup; ++t) {
                if (!((need >> t) & 1)) continue;
                const double *T = tgt[t];
                bool ok = false;
                if (valid && j != ti[t]) {
                    const double r2 = sep2<PERIODIC>(T[0], T[1], T[2], xj, yj, zj, box);
                    const double s = T[3] + hj;
                    ok = r2 < s * s;
                }
                const uint64_t m = __ballot(ok);
                if (ok) {
                    const int64_t pos = (int64_t)cnt[t] + __popcll(m & below);
                    if (pos < A.max_ngb) A.ngb[(int64_t)ta[t] * A.max_ngb + pos] = pj;
                }
                cnt[t] += __popcll(m);
            }
        }
        if (avail < nl) {                       // carry the odd leaf
            const int32_t last = lbuf[nl - 1], lastm = lmsk[nl - 1];
            wave_lds_sync();
            if (lane == 0) { lbuf[0] = last; lmsk[0] = lastm; }
            wave_lds_sync();
        }
        nl -= avail;
        if (sp == 0 && nl == 0) break;
    }
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        if (t < ng && lane == t) {
            A.count[ta[t]] = cnt[t];
            if (cnt[t] > A.max_ngb) atomicOr(A.derr, DERR_NGB_OVERFLOW);
        }
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

hipError_t launch_gather_h(sidm_ctx *c, const double *h_all)
{
    k_gather_h<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, c->perm, h_all, c->hs, c->derr);
    c->hs_valid = 1;
    c->hs_src = h_all;
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
    c->hs_valid = 1;
    c->hs_src = h_all;
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
    const int64_t groups = (n_active + kGroup - 1) / kGroup;
    A.nblk = (groups + kWaves - 1) / kWaves;
    if (A.nblk < 1) A.nblk = 1;
    const unsigned grid = xcd_grid(A.nblk);
    if (c->cfg.periodic) k_overlap<true><<<grid, kBlock, 0, s>>>(A);
    else k_overlap<false><<<grid, kBlock, 0, s>>>(A);
    phase_end(c, PH_OVERLAP);
    return hipGetLastError();
}
