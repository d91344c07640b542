// Tree build for the SIDM neighbour search (the dedicated DM-only tree of the
// paper's sec. 4.3, rebuilt every step on the GPU):
//   bounds -> 48-bit Morton keys -> LSD radix sort (8-bit digits, stable) ->
//   gather of a Morton-ordered structure-of-arrays snapshot ->
//   bucket leaves of SIDM_LEAF consecutive particles -> bottom-up boxes of an
//   implicit binary tree over the leaves.
// Also maps the caller's active list onto Morton order (flag + compaction).
#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

int grid_for(int64_t n, int block = kBlock, int cap = 4096)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

// --- bounds (open boundaries) ------------------------------------------------
__global__ void k_bounds(const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, int64_t n, unsigned long long *bounds)
{
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0, 0, 0};
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long a = ordered_u64(x[t]), b = ordered_u64(y[t]), c = ordered_u64(z[t]);
        mn[0] = min(mn[0], a); mn[1] = min(mn[1], b); mn[2] = min(mn[2], c);
        mx[0] = max(mx[0], a); mx[1] = max(mx[1], b); mx[2] = max(mx[2], c);
    }
    // wave reduction, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        for (int d = 0; d < 3; ++d) {
            mn[d] = min(mn[d], (unsigned long long)__shfl_xor((long long)mn[d], off));
            mx[d] = max(mx[d], (unsigned long long)__shfl_xor((long long)mx[d], off));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        for (int d = 0; d < 3; ++d) {
            atomicMin(&bounds[d], mn[d]);
            atomicMax(&bounds[3 + d], mx[d]);
        }
    }
}

// --- Morton keys ---------------------------------------------------------------
__device__ __forceinline__ uint64_t spread16(uint64_t v)
{
    v &= 0xffffull;
    v = (v | (v << 16)) & 0x0000ff0000ffull;
    v = (v | (v << 8)) & 0x00f00f00f00full;
    v = (v | (v << 4)) & 0x0c30c30c30c3ull;
    v = (v | (v << 2)) & 0x249249249249ull;
    return v;
}

__device__ __forceinline__ uint64_t quant16(double v, double lo, double scale)
{
    double q = (v - lo) * scale;
    if (!(q > 0.0)) return 0;                 // also maps NaN to 0
    if (q >= 65535.0) return 65535;
    return (uint64_t)q;
}

__global__ void k_morton(const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, int64_t n, int periodic, double box,
                         const unsigned long long *__restrict__ bounds, uint64_t *key,
                         int32_t *val)
{
    double lo[3], scale[3];
    for (int d = 0; d < 3; ++d) {
        double l = periodic ? 0.0 : from_ordered_u64(bounds[d]);
        double h = periodic ? box : from_ordered_u64(bounds[3 + d]);
        double ext = h - l;
        lo[d] = l;
        scale[d] = ext > 0.0 ? 65536.0 / ext : 0.0;
    }
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        uint64_t a = quant16(x[t], lo[0], scale[0]);
        uint64_t b = quant16(y[t], lo[1], scale[1]);
        uint64_t c = quant16(z[t], lo[2], scale[2]);
        key[t] = (spread16(a) << 2) | (spread16(b) << 1) | spread16(c);
        val[t] = (int32_t)t;
    }
}

// --- LSD radix sort, 8-bit digits ------------------------------------------------
__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ key, int64_t n,
                                                    int shift, uint32_t *hist, uint32_t *dtot,
                                                    int nblk)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SIDM_SORT_TILE;
    for (int r = 0; r < SIDM_SORT_TILE / 256; ++r) {
        int64_t t = base + r * 256 + threadIdx.x;
        if (t < n) atomicAdd(&cnt[(key[t] >> shift) & 255u], 1u);
    }
    __syncthreads();
    uint32_t c = cnt[threadIdx.x];
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = c;
    if (c) atomicAdd(&dtot[threadIdx.x], c);
}

// one workgroup per digit: exclusive scan over blocks plus the digit's base
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *hist, const uint32_t *dtot, int nblk)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t base_s;
    const int d = blockIdx.x;
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int q = 0; q < d; ++q) b += dtot[q];
        base_s = b;
    }
    uint32_t *h = hist + (int64_t)d * nblk;
    const int per = (nblk + 255) / 256;
    const int lo = threadIdx.x * per;
    uint32_t s = 0;
    for (int q = 0; q < per; ++q) {
        int idx = lo + q;
        if (idx < nblk) s += h[idx];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele over 256 partial sums
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = base_s + (threadIdx.x ? part[threadIdx.x - 1] : 0);
    for (int q = 0; q < per; ++q) {
        int idx = lo + q;
        if (idx < nblk) {
            uint32_t c = h[idx];
            h[idx] = run;
            run += c;
        }
    }
}

// Stable scatter: items are ranked in tile order (round-major, then wave, then lane).
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint64_t *kout, int32_t *vout, int64_t n,
                                                       int shift, const uint32_t *hist, int nblk)
{
    __shared__ uint32_t goff[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    goff[t] = hist[(int64_t)t * nblk + blockIdx.x];
    run[t] = 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * SIDM_SORT_TILE;
    for (int r = 0; r < SIDM_SORT_TILE / 256; ++r) {
        int64_t idx = base + r * 256 + t;
        bool valid = idx < n;
        uint64_t k = valid ? kin[idx] : 0;
        int32_t v = valid ? vin[idx] : 0;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t wrank = __popcll(peers & lt_mask);
        for (int q = 0; q < 4; ++q) wc[q][t] = 0;
        __syncthreads();
        if (valid && wrank == 0) wc[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = goff[d] + run[d] + wrank;
            for (int q = 0; q < w; ++q) pos += wc[q][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        __syncthreads();
    }
}

// --- gather the Morton-ordered snapshot ----------------------------------------------
__global__ void k_gather(int64_t n, const int32_t *__restrict__ order, const double *__restrict__ x,
                         const double *__restrict__ y, const double *__restrict__ z,
                         const double *__restrict__ vx, const double *__restrict__ vy,
                         const double *__restrict__ vz, const double *__restrict__ mass,
                         const uint32_t *__restrict__ id, const uint8_t *__restrict__ st,
                         double *xs, double *ys, double *zs, double *vxs, double *vys, double *vzs,
                         double *ms, uint32_t *ids, uint8_t *sts, int32_t *perm, int32_t *inv)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        int32_t o = order[s];
        xs[s] = x[o]; ys[s] = y[o]; zs[s] = z[o];
        vxs[s] = vx[o]; vys[s] = vy[o]; vzs[s] = vz[o];
        if (mass) ms[s] = mass[o];
        ids[s] = id[o];
        sts[s] = st ? st[o] : (uint8_t)0;
        perm[s] = o;
        inv[o] = (int32_t)s;
    }
}

// --- leaf boxes and bottom-up propagation ----------------------------------------------
__device__ __forceinline__ double load_coherent(const double *p)
{
    unsigned long long b = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(b);
}

__global__ void k_boxes(int64_t n, int64_t p2, const double *__restrict__ xs,
                        const double *__restrict__ ys, const double *__restrict__ zs,
                        double *nodes, int32_t *visit)
{
    int64_t leaf = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (leaf >= p2) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int64_t s0 = leaf * SIDM_LEAF, s1 = s0 + SIDM_LEAF < n ? s0 + SIDM_LEAF : n;
    for (int64_t s = s0; s < s1; ++s) {
        double p[3] = {xs[s], ys[s], zs[s]};
        for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], p[d]); hi[d] = fmax(hi[d], p[d]); }
    }
    int64_t node = p2 + leaf;
    for (int d = 0; d < 3; ++d) { nodes[node * 6 + d] = lo[d]; nodes[node * 6 + 3 + d] = hi[d]; }
    while (node > 1) {
        __threadfence();
        int64_t parent = node >> 1;
        int old = atomicAdd(&visit[parent], 1);
        if (old == 0) return;          // the sibling's thread finishes the parent
        __threadfence();
        const double *a = nodes + (2 * parent) * 6, *b = nodes + (2 * parent + 1) * 6;
        for (int d = 0; d < 3; ++d) {
            nodes[parent * 6 + d] = fmin(load_coherent(a + d), load_coherent(b + d));
            nodes[parent * 6 + 3 + d] = fmax(load_coherent(a + 3 + d), load_coherent(b + 3 + d));
        }
        node = parent;
    }
}

// --- active set -> Morton order --------------------------------------------------------
__global__ void k_mark_active(const int32_t *__restrict__ active, int64_t n_active, int64_t n,
                              const int32_t *__restrict__ inv, int32_t *flag, unsigned int *derr)
{
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n_active;
         a += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = active[a];
        if (i < 0 || i >= n) { atomicOr(derr, DERR_INDEX); continue; }
        int32_t old = atomicExch(&flag[inv[i]], (int32_t)a);
        if (old != -1) atomicOr(derr, DERR_DUPLICATE);
    }
}

__global__ __launch_bounds__(256) void k_count_active(const int32_t *__restrict__ flag, int64_t n,
                                                      int32_t *blk)
{
    __shared__ int32_t part[4];
    int64_t base = (int64_t)blockIdx.x * SIDM_SCAN_TILE;
    int c = 0;
    for (int r = 0; r < SIDM_SCAN_TILE / 256; ++r) {
        int64_t s = base + r * 256 + threadIdx.x;
        c += (s < n && flag[s] >= 0);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// single workgroup: exclusive scan of the per-block counts, total -> *nt
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *blk, int nblk, int32_t *nt)
{
    __shared__ int32_t part[1024];
    const int per = (nblk + 1023) / 1024;
    const int lo = threadIdx.x * per;
    int32_t s = 0;
    for (int q = 0; q < per; ++q)
        if (lo + q < nblk) s += blk[lo + q];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int q = 0; q < per; ++q) {
        if (lo + q < nblk) {
            int32_t c = blk[lo + q];
            blk[lo + q] = run;
            run += c;
        }
    }
    if (threadIdx.x == 1023) *nt = part[1023];
}

__global__ __launch_bounds__(256) void k_compact_active(const int32_t *__restrict__ flag, int64_t n,
                                                        const int32_t *__restrict__ blk,
                                                        int32_t *tlist, int32_t *slot)
{
    __shared__ int32_t wsum[4];
    __shared__ int32_t run_s;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (t == 0) run_s = blk[blockIdx.x];
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SIDM_SCAN_TILE;
    for (int r = 0; r < SIDM_SCAN_TILE / 256; ++r) {
        int64_t s = base + r * 256 + t;
        int32_t f = s < n ? flag[s] : -1;
        bool on = f >= 0;
        uint64_t m = __ballot(on);
        if (lane == 0) wsum[w] = __popcll(m);
        __syncthreads();
        int32_t pos = run_s + __popcll(m & lt_mask);
        for (int q = 0; q < w; ++q) pos += wsum[q];
        if (on) { tlist[pos] = (int32_t)s; slot[pos] = f; }
        __syncthreads();
        if (t == 0) run_s += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_build_tree(sidm_ctx *c, const sidm_particles *p)
{
    hipStream_t s = c->stream;
    const int64_t n = p->n;
    const sidm_config &cfg = c->cfg;
    if (!cfg.periodic) {
        unsigned long long init[6] = {~0ull, ~0ull, ~0ull, 0, 0, 0};
        // tiny fill through a kernel (no memset nodes in captured graphs)
        launch_fill_u64(c->bounds, ~0ull, 3, s);
        launch_fill_u64(c->bounds + 3, 0ull, 3, s);
        (void)init;
        k_bounds<<<grid_for(n, kBlock, 1024), kBlock, 0, s>>>(p->x, p->y, p->z, n, c->bounds);
    }
    k_morton<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, n, cfg.periodic, cfg.box,
                                             c->bounds, c->key0, c->val0);
    const int nblk = (int)((n + SIDM_SORT_TILE - 1) / SIDM_SORT_TILE);
    uint64_t *kin = c->key0, *kout = c->key1;
    int32_t *vin = c->val0, *vout = c->val1;
    for (int shift = 0; shift < 48; shift += 8) {
        launch_fill_i32((int32_t *)c->dtot, 0, 256, s);
        k_radix_hist<<<nblk, 256, 0, s>>>(kin, n, shift, c->hist, c->dtot, nblk);
        k_radix_scan<<<256, 256, 0, s>>>(c->hist, c->dtot, nblk);
        k_radix_scatter<<<nblk, 256, 0, s>>>(kin, vin, kout, vout, n, shift, c->hist, nblk);
        uint64_t *tk = kin; kin = kout; kout = tk;
        int32_t *tv = vin; vin = vout; vout = tv;
    }
    // six passes: the sorted order is back in key0/val0
    k_gather<<<grid_for(n), kBlock, 0, s>>>(n, vin, p->x, p->y, p->z, p->vx, p->vy, p->vz, p->mass,
                                            p->id, p->state, c->xs, c->ys, c->zs, c->vxs, c->vys,
                                            c->vzs, c->ms, c->ids, c->sts, c->perm, c->inv);
    int64_t nleaf = (n + SIDM_LEAF - 1) / SIDM_LEAF;
    int64_t p2 = 1;
    while (p2 < nleaf) p2 <<= 1;
    if (p2 < 2) p2 = 2;
    c->nleaf = nleaf;
    c->p2 = p2;
    launch_fill_i32(c->visit, 0, p2, s);
    k_boxes<<<(int)((p2 + 255) / 256), 256, 0, s>>>(n, p2, c->xs, c->ys, c->zs, c->nodes, c->visit);
    return hipGetLastError();
}

hipError_t launch_map_active(sidm_ctx *c, const int32_t *active, int64_t n_active)
{
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    launch_fill_i32(c->flag, -1, n, s);
    k_mark_active<<<grid_for(n_active), kBlock, 0, s>>>(active, n_active, n, c->inv, c->flag,
                                                        c->derr);
    const int nblk = (int)((n + SIDM_SCAN_TILE - 1) / SIDM_SCAN_TILE);
    k_count_active<<<nblk, 256, 0, s>>>(c->flag, n, c->blk);
    k_scan_blocks<<<1, 1024, 0, s>>>(c->blk, nblk, c->nt_dev);
    k_compact_active<<<nblk, 256, 0, s>>>(c->flag, n, c->blk, c->tlist, c->slot);
    return hipGetLastError();
}
