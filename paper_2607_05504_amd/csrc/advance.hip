// Served form: the step between two scattering steps of an isolated halo.
//
// The paper's SIDM step sits inside a gravity code (sec. 3); a halo served
// here has no gravity solver, so between scattering steps the particles
// move in the fixed potential of a Hernquist (1990) halo,
// Phi(r) = -G M / (r + a), with one kick-drift-kick leapfrog step.  The step
// length is global (one timestep for the whole halo): the largest
// dt_cap / 2^b not above the smallest per-pair bound of the scattering step
// just done (sec. 4.4), so that the next scattering step respects it.
//
//   k_min_dt   block-reduced minimum of dt_sidm into one ordered 64-bit word
//   k_advance  every thread derives the same step length from that word,
//              writes it as the next step's dt of the active particles, and
//              moves its particles: v += g dt/2, x += v dt, v += g dt/2
//   k_drift    a free drift for boxes without gravity (the thermalisation box
//              of sec. 5.2), wrapped into the periodic box
//
// sidm_advance_hernquist_noalloc is the same step for callers that cannot
// allocate: no context, and the reduction's partial minima in a file-scope
// device array (one copy per GPU) instead of context memory.
#include <atomic>

#include "sidm_internal.h"

namespace {

constexpr int kBlock = 256;

int grid_for(int64_t n, int cap = 2048)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

__global__ __launch_bounds__(kBlock) void k_min_dt(const double *__restrict__ dt, int64_t n,
                                                   unsigned long long *out)
{
    __shared__ unsigned long long s_min[kBlock / 64];
    unsigned long long m = ~0ull;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const unsigned long long v = ordered_u64(dt[t]);
        m = v < m ? v : m;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)m, off);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = s_min[w] < m ? s_min[w] : m;
        atomicMin(out, m);
    }
}

// largest dt_cap / 2^b (b = 0..62) not above bound; the smallest one if none is
__device__ __forceinline__ double step_length(double bound, double dt_cap)
{
    double d = dt_cap;
    for (int b = 0; b < 62 && !(d <= bound); ++b) d *= 0.5;
    return d;
}

__global__ __launch_bounds__(kBlock) void k_advance(double *x, double *y, double *z, double *vx,
                                                    double *vy, double *vz, int64_t n,
                                                    int64_t n_active,
                                                    const unsigned long long *minword,
                                                    double dt_cap, double gm, double a,
                                                    double *dt_next, double *dt_step)
{
    const double d = step_length(from_ordered_u64(*minword), dt_cap);
    const double hd = 0.5 * d;
    if (blockIdx.x == 0 && threadIdx.x == 0 && dt_step) *dt_step = d;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        if (t < n_active && dt_next) dt_next[t] = d;
        double px = x[t], py = y[t], pz = z[t];
        double ux = vx[t], uy = vy[t], uz = vz[t];
        // acceleration -G M / (r (r + a)^2) times the position vector
        double r = sqrt((px * px + py * py) + pz * pz);
        double f = r > 0.0 ? -gm / (r * ((r + a) * (r + a))) : 0.0;
        ux += hd * (f * px); uy += hd * (f * py); uz += hd * (f * pz);
        px += d * ux; py += d * uy; pz += d * uz;
        r = sqrt((px * px + py * py) + pz * pz);
        f = r > 0.0 ? -gm / (r * ((r + a) * (r + a))) : 0.0;
        ux += hd * (f * px); uy += hd * (f * py); uz += hd * (f * pz);
        x[t] = px; y[t] = py; z[t] = pz;
        vx[t] = ux; vy[t] = uy; vz[t] = uz;
    }
}

// free drift x += v dt, wrapped into [0, L) in a periodic box
__global__ __launch_bounds__(kBlock) void k_drift(double *x, double *y, double *z,
                                                  const double *__restrict__ vx,
                                                  const double *__restrict__ vy,
                                                  const double *__restrict__ vz, int64_t n,
                                                  double dt, int periodic, double box)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        double p[3] = {x[t] + dt * vx[t], y[t] + dt * vy[t], z[t] + dt * vz[t]};
        if (periodic) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double q = p[d] - box * floor(p[d] / box);
                p[d] = q >= box ? q - box : (q < 0.0 ? 0.0 : q);
            }
        }
        x[t] = p[0]; y[t] = p[1]; z[t] = p[2];
    }
}

// ---------------------------------------------------------------------------
// Allocation-free form: every workgroup of k_min_parts takes kNaPerBlock
// bounds and writes its minimum to scratch[blockIdx.x]; k_min_final reduces
// the partials into scratch[kNaParts]; k_advance reads that word.  Every word
// used is written by the call itself, so nothing needs clearing.
// ---------------------------------------------------------------------------
constexpr int kNaPerThread = 8;
constexpr int64_t kNaPerBlock = (int64_t)kBlock * kNaPerThread;    // 2048 bounds a workgroup
constexpr int kNaParts = 4096;                                    // partial minima at most
constexpr int64_t kNaMaxActive = kNaPerBlock * kNaParts;          // 8,388,608 active particles
constexpr int kNaMaxDevices = 64;
constexpr unsigned long long kOrderedInf = 0xFFF0000000000000ull; // ordered_u64(+inf)

__global__ __launch_bounds__(kBlock) void k_min_parts(const double *__restrict__ dt, int64_t n,
                                                      unsigned long long *parts)
{
    __shared__ unsigned long long s_min[kBlock / 64];
    unsigned long long m = ~0ull;
    const int64_t base = (int64_t)blockIdx.x * kNaPerBlock;
#pragma unroll
    for (int q = 0; q < kNaPerThread; ++q) {
        const int64_t t = base + q * kBlock + threadIdx.x;
        if (t < n) {
            const unsigned long long v = ordered_u64(dt[t]);
            m = v < m ? v : m;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)m, off);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = s_min[w] < m ? s_min[w] : m;
        parts[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_min_final(unsigned long long *parts, int np)
{
    __shared__ unsigned long long s_min[kBlock / 64];
    unsigned long long m = kOrderedInf;
    for (int t = threadIdx.x; t < np; t += kBlock) m = parts[t] < m ? parts[t] : m;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)m, off);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = s_min[w] < m ? s_min[w] : m;
        parts[kNaParts] = m;
    }
}

}  // namespace

// The allocation-free step's scratch: [0, kNaParts) partial minima of the
// bounds, [kNaParts] their minimum.  Each GPU holds its own copy for the
// life of the process; calls on one GPU share it.
static __device__ __align__(256) unsigned long long scratch[kNaParts + 1];

namespace {

// The device address of this GPU's copy of scratch, looked up once per
// device with that device current (the array's name is not a device address
// in host code).
std::atomic<unsigned long long *> g_scratch[kNaMaxDevices];

hipError_t scratch_on_current_device(unsigned long long **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    unsigned long long *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        p = (unsigned long long *)q;
        g_scratch[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return hipSuccess;
}

}  // namespace

extern "C" sidm_status sidm_advance_hernquist_noalloc(void *hip_stream, double *x, double *y,
                                                      double *z, double *vx, double *vy,
                                                      double *vz, int64_t n,
                                                      const double *dt_sidm, int64_t n_active,
                                                      double dt_cap, double gm, double a,
                                                      double *dt_next, double *dt_step)
{
    if (n < 0 || n > (int64_t)INT32_MAX || n_active < 0 || n_active > n) return SIDM_E_INVAL;
    if (n_active > kNaMaxActive) return SIDM_E_CAPACITY;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz)) return SIDM_E_INVAL;
    if (n_active > 0 && !dt_sidm) return SIDM_E_INVAL;
    if (!(dt_cap > 0.0) || !(dt_cap < 1e300) || !(gm >= 0.0) || !(a > 0.0)) return SIDM_E_INVAL;
    if (n == 0) return SIDM_OK;
    unsigned long long *parts = nullptr;
    if (scratch_on_current_device(&parts) != hipSuccess) return SIDM_E_DEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    const int np = (int)((n_active + kNaPerBlock - 1) / kNaPerBlock);
    if (np > 0) k_min_parts<<<np, kBlock, 0, s>>>(dt_sidm, n_active, parts);
    k_min_final<<<1, kBlock, 0, s>>>(parts, np);
    k_advance<<<grid_for(n), kBlock, 0, s>>>(x, y, z, vx, vy, vz, n, n_active, parts + kNaParts,
                                            dt_cap, gm, a, dt_next, dt_step);
    return hipGetLastError() == hipSuccess ? SIDM_OK : SIDM_E_DEVICE;
}

hipError_t launch_drift(sidm_ctx *c, double *x, double *y, double *z, const double *vx,
                        const double *vy, const double *vz, int64_t n, double dt)
{
    k_drift<<<grid_for(n), kBlock, 0, c->stream>>>(x, y, z, vx, vy, vz, n, dt, c->cfg.periodic,
                                                   c->cfg.box);
    return hipGetLastError();
}

hipError_t launch_advance(sidm_ctx *c, double *x, double *y, double *z, double *vx, double *vy,
                          double *vz, int64_t n, const double *dt_sidm, int64_t n_active,
                          double dt_cap, double gm, double a, double *dt_next, double *dt_step)
{
    hipStream_t s = c->stream;
    // the ordered encoding of +inf: with no active particle (or no finite
    // bound) the step is dt_cap itself
    hipError_t e = launch_fill_u64(c->adv_min, 0xFFF0000000000000ull, 1, s);
    if (e != hipSuccess) return e;
    if (n_active > 0) k_min_dt<<<grid_for(n_active), kBlock, 0, s>>>(dt_sidm, n_active, c->adv_min);
    k_advance<<<grid_for(n), kBlock, 0, s>>>(x, y, z, vx, vy, vz, n, n_active, c->adv_min, dt_cap,
                                            gm, a, dt_next, dt_step);
    return hipGetLastError();
}
