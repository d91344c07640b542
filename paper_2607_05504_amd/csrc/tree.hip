// Tree build for the SIDM neighbour search (the dedicated DM-only tree of the
// paper's sec. 4.3, rebuilt every step on the GPU):
//   bounds -> 48-bit Morton keys -> LSD radix sort (8-bit digits, stable) ->
//   the particles packed as 64-byte records and gathered into a Morton-ordered
//   structure-of-arrays snapshot ->
//   bucket leaves of SIDM_LEAF consecutive particles -> boxes of an implicit
//   SIDM_TREE_FAN-ary tree over the leaves, one level per launch.
// Also maps the caller's active list onto Morton order (flag + compaction).
#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;

// Clears, in one launch, the bounding-box accumulators (when the box is
// found from the particles) and the digit totals of the six sort passes.
__global__ void k_tree_reset(unsigned long long *bounds, int clear_bounds, uint32_t *dtot, int ndtot)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (clear_bounds && t < 6) bounds[t] = t < 3 ? ~0ull : 0ull;
    if (t < ndtot) dtot[t] = 0u;
}

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
__global__ __launch_bounds__(256) void k_bounds(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z, int64_t n,
                                                unsigned long long *bounds)
{
    __shared__ unsigned long long part[4][6];
    unsigned long long v[6] = {~0ull, ~0ull, ~0ull, 0, 0, 0};
    auto take = [&](double px, double py, double pz) {
        const unsigned long long a = ordered_u64(px), b = ordered_u64(py), c = ordered_u64(pz);
        v[0] = min(v[0], a); v[1] = min(v[1], b); v[2] = min(v[2], c);
        v[3] = max(v[3], a); v[4] = max(v[4], b); v[5] = max(v[5], c);
    };
    // four particles a thread per round, their positions requested together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; t + 3 * stride < n; t += 4 * stride) {
        double px[4], py[4], pz[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            px[u] = x[t + u * stride]; py[u] = y[t + u * stride]; pz[u] = z[t + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) take(px[u], py[u], pz[u]);
    }
    for (; t < n; t += stride) take(x[t], y[t], z[t]);
    for (int off = 32; off > 0; off >>= 1) {
        for (int d = 0; d < 3; ++d) {
            v[d] = min(v[d], (unsigned long long)__shfl_xor((long long)v[d], off));
            v[3 + d] = max(v[3 + d], (unsigned long long)__shfl_xor((long long)v[3 + d], off));
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 6; ++d) part[w][d] = v[d];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        unsigned long long r = part[0][d];
        for (int q = 1; q < 4; ++q) r = d < 3 ? min(r, part[q][d]) : max(r, part[q][d]);
        if (d < 3) atomicMin(&bounds[d], r); else atomicMax(&bounds[d], r);
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

// Keys of one sort tile per workgroup, with the digit counts the sort needs:
// the totals of every 8-bit digit of every pass into dtot[pass * 256 + digit]
// (they do not depend on the keys' order; dtot must start at zero), and this
// tile's counts of the first pass's digits into hist[digit * nblk + tile].
__global__ __launch_bounds__(256) void k_morton(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z, int64_t n,
                                                int periodic, double box,
                                                const unsigned long long *__restrict__ bounds,
                                                uint64_t *key, int32_t *val, uint32_t *dtot,
                                                uint32_t *hist, int nblk)
{
    __shared__ uint32_t cnt[6 * 256];
    for (int q = threadIdx.x; q < 6 * 256; q += 256) cnt[q] = 0;
    double lo[3], scale[3];
    for (int d = 0; d < 3; ++d) {
        double l = periodic ? 0.0 : from_ordered_u64(bounds[d]);
        double h = periodic ? box : from_ordered_u64(bounds[3 + d]);
        double ext = h - l;
        lo[d] = l;
        scale[d] = ext > 0.0 ? 65536.0 / ext : 0.0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SIDM_SORT_TILE;
    for (int r = 0; r < SIDM_SORT_TILE / 256; ++r) {
        const int64_t t = base + r * 256 + threadIdx.x;
        if (t >= n) break;
        uint64_t a = quant16(x[t], lo[0], scale[0]);
        uint64_t b = quant16(y[t], lo[1], scale[1]);
        uint64_t c = quant16(z[t], lo[2], scale[2]);
        const uint64_t k = (spread16(a) << 2) | (spread16(b) << 1) | spread16(c);
        key[t] = k;
        val[t] = (int32_t)t;
#pragma unroll
        for (int p = 0; p < 6; ++p) atomicAdd(&cnt[p * 256 + ((k >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
    for (int q = threadIdx.x; q < 6 * 256; q += 256)
        if (cnt[q]) atomicAdd(&dtot[q], cnt[q]);
}

// --- LSD radix sort, 8-bit digits ------------------------------------------------
__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ key, int64_t n,
                                                    int shift, uint32_t *hist, int nblk)
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
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// one workgroup per digit: exclusive scan over blocks plus the digit's base
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *hist, const uint32_t *dtot, int nblk)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t dsum[256];
    const int d = blockIdx.x;
    // the digit's base: exclusive prefix of the digit totals
    dsum[threadIdx.x] = dtot[threadIdx.x];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? dsum[threadIdx.x - off] : 0;
        __syncthreads();
        dsum[threadIdx.x] += v;
        __syncthreads();
    }
    const uint32_t base_s = d ? dsum[d - 1] : 0u;
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

// Stable scatter: items are ranked in tile order (round-major, then wave,
// then lane) within their digit.  The tile is first reordered by digit in LDS
// and then written out, so a digit's items go to consecutive addresses.  The
// last pass (perm != NULL) writes the index maps instead of keys and values:
// perm[pos] = the caller index that lands at pos, inv[that index] = pos.
constexpr int kRounds = SIDM_SORT_TILE / 256;

__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint64_t *kout, int32_t *vout, int64_t n,
                                                       int shift, const uint32_t *hist, int nblk,
                                                       int32_t *perm, int32_t *inv)
{
    __shared__ uint32_t goff[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    __shared__ uint64_t s_key[SIDM_SORT_TILE];
    __shared__ int32_t s_val[SIDM_SORT_TILE];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    goff[t] = hist[(int64_t)t * nblk + blockIdx.x];
    run[t] = 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * SIDM_SORT_TILE;
    uint64_t kk[kRounds];
    int32_t vv[kRounds];
    uint32_t rk[kRounds];                      // rank within the digit in the tile
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t idx = base + r * 256 + t;
        const bool valid = idx < n;
        const uint64_t k = valid ? kin[idx] : 0;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        kk[r] = k;
        vv[r] = valid ? vin[idx] : 0;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t wrank = __popcll(peers & lt_mask);
        for (int q = 0; q < 4; ++q) wc[q][t] = 0;
        __syncthreads();
        if (valid && wrank == 0) wc[w][d] = __popcll(peers);
        __syncthreads();
        uint32_t pos = run[d] + wrank;
        for (int q = 0; q < w; ++q) pos += wc[q][d];
        rk[r] = valid ? pos : 0xffffffffu;
        __syncthreads();
        run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        __syncthreads();
    }
    // run[d] now counts the tile's items of digit d: exclusive prefix = where
    // digit d starts in the tile (Hillis-Steele in wc[0], wc[1])
    uint32_t *sa = wc[0], *sb = wc[1];
    sa[t] = run[t];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        sb[t] = sa[t] + (t >= off ? sa[t - off] : 0u);
        __syncthreads();
        uint32_t *tmp = sa; sa = sb; sb = tmp;
    }
    const uint32_t start_t = sa[t] - run[t];   // exclusive prefix of digit t
    __syncthreads();
    wc[2][t] = start_t;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (rk[r] != 0xffffffffu) {
            const uint32_t d = (uint32_t)(kk[r] >> shift) & 255u;
            const uint32_t lp = wc[2][d] + rk[r];
            s_key[lp] = kk[r];
            s_val[lp] = vv[r];
        }
    }
    __syncthreads();
    const int64_t cnt = n - base < SIDM_SORT_TILE ? n - base : SIDM_SORT_TILE;
    for (int i = t; i < cnt; i += 256) {
        const uint64_t k = s_key[i];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = goff[d] + (uint32_t)i - wc[2][d];
        if (perm) {
            const int32_t o = s_val[i];
            perm[pos] = o;
            inv[o] = (int32_t)pos;
        } else {
            kout[pos] = k;
            vout[pos] = s_val[i];
        }
    }
}

// --- the Morton-ordered snapshot ------------------------------------------------------
// The snapshot in two passes.  k_pack writes each caller particle as one
// 64-byte record (x y z vx vy vz m, id | state << 32), reading the caller's
// arrays in their order; k_gather_rec then fills sorted slot s from record
// perm[s], four lanes a record (16 bytes each, one 64-byte segment), and
// writes the sorted arrays coalesced.  One random access a particle instead
// of one for each of its nine arrays.
__global__ __launch_bounds__(256) void k_pack(int64_t n, const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const double *__restrict__ vx,
                                              const double *__restrict__ vy,
                                              const double *__restrict__ vz,
                                              const double *__restrict__ mass,
                                              const uint32_t *__restrict__ id,
                                              const uint8_t *__restrict__ st, double2 *rec)
{
    // a lane a 16-byte quarter of a record: consecutive lanes write
    // consecutive bytes
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 4 * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = t >> 2;
        const int q = (int)(t & 3);
        double2 v;
        if (q < 3) {
            const double *pa = q == 0 ? x : q == 1 ? z : vy;
            const double *pb = q == 0 ? y : q == 1 ? vx : vz;
            v = make_double2(pa[o], pb[o]);
        } else {
            const uint64_t w = (uint64_t)id[o] | ((uint64_t)(st ? st[o] : 0) << 32);
            v = make_double2(mass ? mass[o] : 0.0, __longlong_as_double((long long)w));
        }
        rec[t] = v;
    }
}

__global__ __launch_bounds__(256) void k_gather_rec(int64_t n, const int32_t *__restrict__ perm,
                                                    const double2 *__restrict__ rec, int has_mass,
                                                    double *xs, double *ys, double *zs,
                                                    double *vxs, double *vys, double *vzs,
                                                    double *ms, uint32_t *ids, uint8_t *sts)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 4 * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = t >> 2;
        const int q = (int)(t & 3);
        const double2 v = rec[(int64_t)perm[s] * 4 + q];
        if (q == 0) {
            xs[s] = v.x; ys[s] = v.y;
        } else if (q == 1) {
            zs[s] = v.x; vxs[s] = v.y;
        } else if (q == 2) {
            vys[s] = v.x; vzs[s] = v.y;
        } else {
            if (has_mass) ms[s] = v.x;
            const uint64_t w = (uint64_t)__double_as_longlong(v.y);
            ids[s] = (uint32_t)w;
            sts[s] = (uint8_t)(w >> 32);
        }
    }
}

// --- bucket tree boxes --------------------------------------------------------------
// Two leaves per wavefront: lane l holds particle (leaf*32 + l%32); min/max by
// butterfly shuffles within each half-wave, over the 8 lanes of a sub-bucket
// first (its box is written in FP32 rounded outward, so that it contains the
// exact box), then over the leaf.  A workgroup's 8 leaves are the children of
// one level-1 node, whose box it writes too (at nodes[off1 + b]).
__global__ __launch_bounds__(256) void k_leaf_boxes(int64_t n, int64_t nleaf,
                                                    const double *__restrict__ xs,
                                                    const double *__restrict__ ys,
                                                    const double *__restrict__ zs, double *nodes,
                                                    float *sbox, int64_t off1, int64_t cnt1)
{
    static_assert(SIDM_TREE_FAN * SIDM_LEAF == 256, "a workgroup covers one level-1 node");
    static_assert(SIDM_SUB == 8, "a sub-bucket box is 8 floats, one per lane");
    __shared__ double s_box[SIDM_TREE_FAN][6];
    const int64_t leaf = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
    const int sub = threadIdx.x & 31;
    const int64_t s = leaf * SIDM_LEAF + sub;
    const bool in = leaf < nleaf && s < n;
    double v[6];
    if (in) {
        v[0] = v[3] = xs[s];
        v[1] = v[4] = ys[s];
        v[2] = v[5] = zs[s];
    } else {
        v[0] = v[1] = v[2] = INFINITY;
        v[3] = v[4] = v[5] = -INFINITY;
    }
    for (int off = 1; off < 32; off <<= 1) {
        if (off == SIDM_SUB && leaf < nleaf) {
            // lane d of the sub-bucket writes float d of its box
            const int d = sub % SIDM_SUB;
            float f = 0.0f;
            if (d < 3) f = __double2float_rd(v[d]);
            else if (d >= 4 && d < 7) f = __double2float_ru(v[d - 1]);
            sbox[(leaf * (SIDM_LEAF / SIDM_SUB) + sub / SIDM_SUB) * 8 + d] = f;
        }
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], __shfl_xor(v[d], off));
            v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], off));
        }
    }
    if (sub < 6) {
        if (leaf < nleaf) nodes[leaf * 6 + sub] = v[sub];
        s_box[threadIdx.x >> 5][sub] = v[sub];     // an empty box past the last leaf
    }
    __syncthreads();
    if (threadIdx.x < 6 && (int64_t)blockIdx.x < cnt1) {
        const int d = threadIdx.x;
        double r = s_box[0][d];
        for (int c = 1; c < SIDM_TREE_FAN; ++c) r = d < 3 ? fmin(r, s_box[c][d]) : fmax(r, s_box[c][d]);
        nodes[(off1 + blockIdx.x) * 6 + d] = r;
    }
}

// The small upper levels in one workgroup, level after level from `from`.
__global__ __launch_bounds__(1024) void k_top_levels(double *nodes, TreeLevels lv, int from)
{
    for (int l = from; l < lv.nlev; ++l) {
        const int64_t off_child = lv.off[l - 1], cnt_child = lv.cnt[l - 1];
        for (int64_t q = threadIdx.x; q < lv.cnt[l]; q += 1024) {
            double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            for (int c = 0; c < SIDM_TREE_FAN; ++c) {
                const int64_t ch = q * SIDM_TREE_FAN + c;
                if (ch >= cnt_child) break;
                const double *b = nodes + (off_child + ch) * 6;
                for (int d = 0; d < 3; ++d) {
                    v[d] = fmin(v[d], b[d]);
                    v[3 + d] = fmax(v[3 + d], b[3 + d]);
                }
            }
            for (int d = 0; d < 6; ++d) nodes[(lv.off[l] + q) * 6 + d] = v[d];
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Boxes of level l from the boxes of level l-1 (one thread per node).
__global__ void k_level_boxes(double *nodes, int64_t off_child, int64_t cnt_child, int64_t off,
                              int64_t cnt)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < SIDM_TREE_FAN; ++c) {
        const int64_t ch = q * SIDM_TREE_FAN + c;
        if (ch >= cnt_child) break;
        const double *b = nodes + (off_child + ch) * 6;
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], b[d]);
            v[3 + d] = fmax(v[3 + d], b[3 + d]);
        }
    }
    for (int d = 0; d < 6; ++d) nodes[(off + q) * 6 + d] = v[d];
}

// --- active set -> Morton order --------------------------------------------------------
// Plain stores mark the sorted slots (a duplicate entry overwrites its twin);
// the entries out of range are counted in *bad, so that the scan finds a
// duplicate as fewer marked slots than valid entries.
__global__ void k_mark_active(const int32_t *__restrict__ active, int64_t n_active, int64_t n,
                              const int32_t *__restrict__ inv, int32_t *flag, int32_t *bad,
                              unsigned int *derr)
{
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n_active;
         a += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = active[a];
        if (i < 0 || i >= n) {
            atomicOr(derr, DERR_INDEX);
            atomicAdd(bad, 1);
            continue;
        }
        flag[inv[i]] = (int32_t)a;
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

// single workgroup: exclusive scan of the per-block counts, total -> *nt;
// blk[nblk] holds the active entries out of range: fewer marked slots than
// the other entries means a duplicate
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *blk, int nblk, int32_t *nt, int64_t n_active,
                                                      unsigned int *derr)
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
    if (threadIdx.x == 1023) {
        *nt = part[1023];
        if ((int64_t)part[1023] + blk[nblk] < n_active) atomicOr(derr, DERR_DUPLICATE);
    }
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

// Mixed form: each particle's offset from its leaf's box centre, in FP32.
__global__ __launch_bounds__(256) void k_leaf_offsets(int64_t n, const double *__restrict__ xs,
                                                      const double *__restrict__ ys,
                                                      const double *__restrict__ zs,
                                                      const double *__restrict__ nodes, float *xo,
                                                      float *yo, float *zo)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double *b = nodes + (j / SIDM_LEAF) * 6;
        xo[j] = (float)(xs[j] - box_centre(b, 0));
        yo[j] = (float)(ys[j] - box_centre(b, 1));
        zo[j] = (float)(zs[j] - box_centre(b, 2));
    }
}


hipError_t launch_build_tree(sidm_ctx *c, const sidm_particles *p)
{
    hipStream_t s = c->stream;
    const int64_t n = p->n;
    const sidm_config &cfg = c->cfg;
    // tiny clears through a kernel (no memset nodes in captured graphs)
    k_tree_reset<<<(6 * 256 + kBlock - 1) / kBlock, kBlock, 0, s>>>(c->bounds, cfg.periodic ? 0 : 1,
                                                                   c->dtot, 6 * 256);
    if (!cfg.periodic)
        k_bounds<<<grid_for(n, kBlock, 256), kBlock, 0, s>>>(p->x, p->y, p->z, n, c->bounds);
    const int nblk = (int)((n + SIDM_SORT_TILE - 1) / SIDM_SORT_TILE);
    k_morton<<<nblk, 256, 0, s>>>(p->x, p->y, p->z, n, cfg.periodic, cfg.box, c->bounds, c->key0,
                                  c->val0, c->dtot, c->hist, nblk);
    uint64_t *kin = c->key0, *kout = c->key1;
    int32_t *vin = c->val0, *vout = c->val1;
    for (int shift = 0; shift < 48; shift += 8) {
        if (shift > 0) k_radix_hist<<<nblk, 256, 0, s>>>(kin, n, shift, c->hist, nblk);
        k_radix_scan<<<256, 256, 0, s>>>(c->hist, c->dtot + (shift / 8) * 256, nblk);
        const bool last = shift == 40;
        k_radix_scatter<<<nblk, 256, 0, s>>>(kin, vin, kout, vout, n, shift, c->hist, nblk,
                                             last ? c->perm : nullptr, last ? c->inv : nullptr);
        uint64_t *tk = kin; kin = kout; kout = tk;
        int32_t *tv = vin; vin = vout; vout = tv;
    }
    // the last of the six passes wrote perm and inv
    return launch_refit_tree(c, p);
}

// Snapshot in the order of the last sort, then the boxes bottom-up.  Alone
// (sidm_refit_tree) it reuses that order for particles that have moved: the
// boxes are those of the current positions, so searches stay exact; only the
// tree's tightness degrades as the order ages.
hipError_t launch_refit_tree(sidm_ctx *c, const sidm_particles *p)
{
    hipStream_t s = c->stream;
    const int64_t n = p->n;
    const sidm_config &cfg = c->cfg;
    k_pack<<<grid_for(4 * n), kBlock, 0, s>>>(n, p->x, p->y, p->z, p->vx, p->vy, p->vz, p->mass, p->id,
                                         p->state, (double2 *)c->rec);
    k_gather_rec<<<grid_for(4 * n), kBlock, 0, s>>>(n, c->perm, (const double2 *)c->rec,
                                                    p->mass != nullptr, c->xs, c->ys, c->zs,
                                                    c->vxs, c->vys, c->vzs, c->ms, c->ids, c->sts);
    c->lv = tree_levels(n);
    const TreeLevels &lv = c->lv;
    const int64_t nleaf = lv.cnt[0];
    // leaves and level 1 together, then the big levels one launch each, then
    // the small ones in a single workgroup
    k_leaf_boxes<<<(unsigned)((nleaf * 32 + 255) / 256), 256, 0, s>>>(
        n, nleaf, c->xs, c->ys, c->zs, c->nodes, c->sbox, lv.off[1], lv.cnt[1]);
    int l = 2;
    for (; l < lv.nlev && lv.cnt[l] > 1024; ++l)
        k_level_boxes<<<(unsigned)((lv.cnt[l] + 255) / 256), 256, 0, s>>>(
            c->nodes, lv.off[l - 1], lv.cnt[l - 1], lv.off[l], lv.cnt[l]);
    if (l < lv.nlev) k_top_levels<<<1, 1024, 0, s>>>(c->nodes, lv, l);
    if (cfg.precision == SIDM_MIXED)
        k_leaf_offsets<<<grid_for(n), kBlock, 0, s>>>(n, c->xs, c->ys, c->zs, c->nodes, c->xo,
                                                      c->yo, c->zo);
    return hipGetLastError();
}

hipError_t launch_map_active(sidm_ctx *c, const int32_t *active, int64_t n_active)
{
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    phase_begin(c, PH_MAP);
    const int nblk = (int)((n + SIDM_SCAN_TILE - 1) / SIDM_SCAN_TILE);
    launch_fill_i32(c->flag, -1, n, s);
    launch_fill_i32(c->blk + nblk, 0, 1, s);
    k_mark_active<<<grid_for(n_active), kBlock, 0, s>>>(active, n_active, n, c->inv, c->flag,
                                                        c->blk + nblk, c->derr);
    k_count_active<<<nblk, 256, 0, s>>>(c->flag, n, c->blk);
    k_scan_blocks<<<1, 1024, 0, s>>>(c->blk, nblk, c->nt_dev, n_active, c->derr);
    k_compact_active<<<nblk, 256, 0, s>>>(c->flag, n, c->blk, c->tlist, c->slot);
    phase_end(c, PH_MAP);
    return hipGetLastError();
}
