// Exact N_ngb-nearest-neighbour search of the active particles (paper sec. 4.2
// and 4.5: h_i is set so that N_ngb neighbours lie inside the kernel; here
// exactly N_ngb, ties broken by particle ID, h_i = distance of the next one).
//
// One wavefront serves 64 Morton-consecutive targets, one per lane (the
// paper's grouped walk for four particles, sec. 4.3, widened to a wavefront):
// the wave walks the bucket tree once, opening a node if any lane needs it, and
// every lane ranks every particle of every opened leaf.  Each lane keeps the
// n_ngb + 1 best (r^2, id) seen so far in a max-heap in LDS; its root is the
// lane's pruning radius.  Node tests are exact-conservative: the gap to a box
// is computed with the same rounded operations as a candidate's separation,
// and rounding is monotone, so no candidate with r^2 <= the radius is pruned.
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
    int64_t n, p2;
    int k;
    double box;
};

// gap along one axis between the lane's point p and a box [lo, hi], as the
// candidates would compute it (min over the periodic images)
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

// per-axis image shift valid for every particle of a box, or NaN if mixed
template <bool PERIODIC>
__device__ __forceinline__ double axis_shift(double lo, double hi, double p, double box)
{
    if (!PERIODIC) return 0.0;
    double a = lo - p, b = hi - p, half = 0.5 * box;
    if (a >= half) return -box;
    if (b < -half) return box;
    if (a >= -half && b < half) return 0.0;
    return __longlong_as_double(0x7ff8000000000000ll);
}

// heap entry e of this lane lives at [e * 64 + lane]
struct LaneHeap {
    double *r2;
    int32_t *j;
    int lane;
    __device__ double &R(int e) { return r2[e * 64 + lane]; }
    __device__ int32_t &J(int e) { return j[e * 64 + lane]; }
};

// (r2a, ja) > (r2b, jb) by (r^2, id)
__device__ __forceinline__ bool key_gt(double r2a, int32_t ja, double r2b, int32_t jb,
                                       const uint32_t *__restrict__ ids)
{
    if (r2a != r2b) return r2a > r2b;
    return ids[ja] > ids[jb];
}

__device__ __forceinline__ void sift_down(LaneHeap &H, int pos, int size, double r2, int32_t j,
                                          const uint32_t *__restrict__ ids)
{
    while (true) {
        int c = 2 * pos + 1;
        if (c >= size) break;
        double cr = H.R(c);
        int32_t cj = H.J(c);
        if (c + 1 < size) {
            double c2r = H.R(c + 1);
            int32_t c2j = H.J(c + 1);
            if (key_gt(c2r, c2j, cr, cj, ids)) { c = c + 1; cr = c2r; cj = c2j; }
        }
        if (!key_gt(cr, cj, r2, j, ids)) break;
        H.R(pos) = cr;
        H.J(pos) = cj;
        pos = c;
    }
    H.R(pos) = r2;
    H.J(pos) = j;
}

template <bool PERIODIC, int K1MAX>
__global__ __launch_bounds__(64) void k_knn(KnnArgs A)
{
    __shared__ double s_r2[K1MAX * 64];
    __shared__ int32_t s_j[K1MAX * 64];
    __shared__ int32_t s_stack[96];

    const int nt = *A.nt_dev;
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    if (b0 >= nt) return;
    const int lane = threadIdx.x;
    const int64_t b = b0 + lane;
    const bool valid = b < nt;
    const int32_t i = A.tlist[valid ? b : nt - 1];
    const double px = A.xs[i], py = A.ys[i], pz = A.zs[i];
    const int K1 = A.k + 1;
    const double box = A.box;
    const uint32_t *__restrict__ ids = A.ids;

    LaneHeap H{s_r2, s_j, lane};
    int cnt = 0;
    double T = INFINITY;        // r^2 of the heap root once full
    int32_t Tj = -1;

    // reference point for near-first child order: the wave's first target
    const double rx = __shfl(px, 0), ry = __shfl(py, 0), rz = __shfl(pz, 0);

    int sp = 1;
    s_stack[0] = 1;
    while (sp > 0) {
        --sp;
        const int64_t node = __builtin_amdgcn_readfirstlane(s_stack[sp]);
        const double *nb = A.nodes + node * 6;
        const double lx = nb[0], ly = nb[1], lz = nb[2], hx = nb[3], hy = nb[4], hz = nb[5];
        if (!(lx <= hx)) continue;   // empty box
        double gx = axis_gap<PERIODIC>(lx, hx, px, box);
        double gy = axis_gap<PERIODIC>(ly, hy, py, box);
        double gz = axis_gap<PERIODIC>(lz, hz, pz, box);
        double d2 = (gx * gx + gy * gy) + gz * gz;
        bool need = valid && (cnt < K1 || d2 <= T);
        if (!__any(need)) continue;
        if (node >= A.p2) {
            // leaf: particles [s0, s0 + m) of the Morton-ordered snapshot
            const int64_t s0 = (node - A.p2) * SIDM_LEAF;
            const int m = (int)((A.n - s0) < SIDM_LEAF ? (A.n - s0) : SIDM_LEAF);
            double sx = axis_shift<PERIODIC>(lx, hx, px, box);
            double sy = axis_shift<PERIODIC>(ly, hy, py, box);
            double sz = axis_shift<PERIODIC>(lz, hz, pz, box);
            bool mixed = PERIODIC && (isnan(sx) || isnan(sy) || isnan(sz));
            const bool any_mixed = __any(mixed);
            for (int c = 0; c < m; ++c) {
                const int32_t j = (int32_t)(s0 + c);
                const double qx = A.xs[j], qy = A.ys[j], qz = A.zs[j];
                double r2;
                if (!PERIODIC) {
                    double dx = qx - px, dy = qy - py, dz = qz - pz;
                    r2 = (dx * dx + dy * dy) + dz * dz;
                } else if (!any_mixed) {
                    // same rounding as the wrapped separation: d + 0 == d, d + (-L) == d - L
                    double dx = (qx - px) + sx, dy = (qy - py) + sy, dz = (qz - pz) + sz;
                    r2 = (dx * dx + dy * dy) + dz * dz;
                } else {
                    r2 = sep2<true>(px, py, pz, qx, qy, qz, box);
                }
                if (!valid || j == i) continue;
                if (cnt < K1) {
                    H.R(cnt) = r2;
                    H.J(cnt) = j;
                    ++cnt;
                    if (cnt == K1) {
                        for (int e = K1 / 2 - 1; e >= 0; --e) sift_down(H, e, K1, H.R(e), H.J(e), ids);
                        T = H.R(0);
                        Tj = H.J(0);
                    }
                } else if (r2 < T || (r2 == T && ids[j] < ids[Tj])) {
                    sift_down(H, 0, K1, r2, j, ids);
                    T = H.R(0);
                    Tj = H.J(0);
                }
            }
        } else {
            // push the far child first so the near one is walked next
            const int64_t c0 = 2 * node, c1 = 2 * node + 1;
            const double *n0 = A.nodes + c0 * 6, *n1 = A.nodes + c1 * 6;
            double e0x = 0.5 * (n0[0] + n0[3]) - rx, e0y = 0.5 * (n0[1] + n0[4]) - ry,
                   e0z = 0.5 * (n0[2] + n0[5]) - rz;
            double e1x = 0.5 * (n1[0] + n1[3]) - rx, e1y = 0.5 * (n1[1] + n1[4]) - ry,
                   e1z = 0.5 * (n1[2] + n1[5]) - rz;
            double q0 = e0x * e0x + e0y * e0y + e0z * e0z;
            double q1 = e1x * e1x + e1y * e1y + e1z * e1z;
            bool near0 = !(q1 < q0);
            s_stack[sp] = (int32_t)(near0 ? c1 : c0);
            s_stack[sp + 1] = (int32_t)(near0 ? c0 : c1);
            sp += 2;
        }
    }

    if (!valid) return;
    if (cnt < K1) {
        atomicOr(A.derr, DERR_COUNT);
        return;
    }
    // heap sort: ascending (r^2, id) in entries 0..K1-1
    for (int end = K1 - 1; end > 0; --end) {
        double r = H.R(end);
        int32_t jj = H.J(end);
        H.R(end) = H.R(0);
        H.J(end) = H.J(0);
        sift_down(H, 0, end, r, jj, ids);
    }
    const int32_t a = A.slot[b];
    A.h[a] = sqrt(H.R(K1 - 1));
    int32_t *out = A.ngb + (int64_t)a * A.k;
    for (int s = 0; s < A.k; ++s) out[s] = A.perm[H.J(s)];
}

template <bool P, int K1MAX>
void launch_one(const KnnArgs &A, int64_t n_active, hipStream_t s)
{
    int64_t blocks = (n_active + 63) / 64;
    k_knn<P, K1MAX><<<(unsigned)blocks, 64, 0, s>>>(A);
}

}  // namespace

hipError_t launch_knn(sidm_ctx *c, int64_t n_active, int32_t *ngb, double *h)
{
    KnnArgs A;
    A.xs = c->xs; A.ys = c->ys; A.zs = c->zs;
    A.ids = c->ids; A.perm = c->perm; A.nodes = c->nodes;
    A.tlist = c->tlist; A.slot = c->slot; A.nt_dev = c->nt_dev;
    A.ngb = ngb; A.h = h; A.derr = c->derr;
    A.n = c->n; A.p2 = c->p2; A.k = c->cfg.n_ngb; A.box = c->cfg.box;
    const bool per = c->cfg.periodic != 0;
    const int k1 = A.k + 1;
    if (k1 <= 17) {
        per ? launch_one<true, 17>(A, n_active, c->stream) : launch_one<false, 17>(A, n_active, c->stream);
    } else if (k1 <= 33) {
        per ? launch_one<true, 33>(A, n_active, c->stream) : launch_one<false, 33>(A, n_active, c->stream);
    } else {
        per ? launch_one<true, 65>(A, n_active, c->stream) : launch_one<false, 65>(A, n_active, c->stream);
    }
    return hipGetLastError();
}
