// Radius-independent kernels (model set-up, multi-source injection, streaming
// bandwidth reference) and the registry/launchers over the per-radius objects.
#include "internal.h"

namespace p1310 {

const ZVariant *zmarch_table_r3(int *n);
const ZVariant *zmarch_table_r4(int *n);
const ZVariant *zmarch_table_r5(int *n);
const Z2Variant *zmarch2_table_r3(int *n);
const Z2Variant *zmarch2_table_r4(int *n);
const Z2Variant *zmarch2_table_r5(int *n);
hipError_t launch_plain_r3(int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s);
hipError_t launch_plain_r4(int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s);
hipError_t launch_plain_r5(int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s);

namespace {

struct Registry {
    const ZVariant *items[256];
    int n = 0;
    Registry()
    {
        const ZVariant *(*tables[])(int *) = {zmarch_table_r3, zmarch_table_r4, zmarch_table_r5};
        for (auto f : tables) {
            int k = 0;
            const ZVariant *t = f(&k);
            for (int i = 0; i < k && n < 256; ++i) items[n++] = &t[i];
        }
    }
};

const Registry &registry()
{
    static Registry r;
    return r;
}

struct Registry2 {
    const Z2Variant *items[64];
    int n = 0;
    Registry2()
    {
        const Z2Variant *(*tables[])(int *) = {zmarch2_table_r3, zmarch2_table_r4, zmarch2_table_r5};
        for (auto f : tables) {
            int k = 0;
            const Z2Variant *t = f(&k);
            for (int i = 0; i < k && n < 64; ++i) items[n++] = &t[i];
        }
    }
};

const Registry2 &registry2()
{
    static Registry2 r;
    return r;
}

// kappa = (v dt / h)^2 formed in FP64, rounded once to FP32.
__global__ void __launch_bounds__(256) kappa_kernel(const float *v, float *kappa, int64_t n, double dt, double h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double r = (double)v[i] * dt / h;
        kappa[i] = (float)(r * r);
    }
}

// kappa = dt^2 / (h^2 m) from squared slowness m = 1/v^2, in FP64, rounded once.
__global__ void __launch_bounds__(256) kappa_m_kernel(const float *m, float *kappa, int64_t n, double dt, double h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double num = dt * dt / (h * h);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        kappa[i] = (float)(num / (double)m[i]);
}

// Several point sources, one thread per source. Repeated indices are added
// by the thread of their first occurrence, in index order, so the result is
// the same as adding the sources one after another. Finding repeats: every
// workgroup walks the index list in chunks of kInjectChunk and builds, in
// LDS, a hash table (linear probing) from grid index to the first and last
// source number and the number of occurrences in the chunk; each thread then
// looks up its own index. A chunk before the thread's own that holds the
// index, or a first occurrence before the thread in its own chunk, makes an
// earlier thread the owner. The owner adds its chunk's occurrences and those
// of later chunks in order: the one or two positions the table names, or a
// scan from the first to the last when a chunk holds the index three or more
// times. Cost: O(n / 256) LDS atomics per thread and chunk, instead of the
// O(n) dependent reads of a direct search.
constexpr int kInjectChunk = 1024;               // source indices per chunk
constexpr int kInjectSlots = 2 * kInjectChunk;   // hash table capacity (power of two)

__device__ __forceinline__ uint32_t inject_slot(uint64_t q, uint32_t mask)
{
    return (uint32_t)((q * 0x9E3779B97F4A7C15ull) >> 40) & mask;  // Fibonacci hashing
}

template <typename ST>
__global__ void __launch_bounds__(256) inject_kernel(ST *u, const float *kappa, int64_t n_points, int64_t pitch,
                                                     int64_t nx, const int64_t *idx, const float *amp, int nsrc,
                                                     int64_t it, float scale)
{
    // A grid point: inside the array and not in a row's padding.
    auto on_grid = [&](int64_t q) { return q >= 0 && q < n_points && (pitch == nx || q % pitch < nx); };
    __shared__ unsigned long long keys[kInjectSlots];
    __shared__ int kfirst[kInjectSlots], klast[kInjectSlots], kcount[kInjectSlots];
    const unsigned long long kEmpty = ~0ull;  // no grid index (they are >= 0)
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = j < nsrc ? idx[j] : -1;
    bool owner = on_grid(p);
    float kp = 0.0f, v = 0.0f;
    if (owner) {
        kp = kappa[p];
        v = (float)u[p];
    }
    const float *row = amp + it * nsrc;
    for (int c0 = 0; c0 < nsrc; c0 += kInjectChunk) {
        const int cn = min(kInjectChunk, nsrc - c0);
        int H = 64;
        while (H < 2 * cn) H *= 2;
        const uint32_t mask = (uint32_t)H - 1;
        __syncthreads();  // the previous chunk's lookups are done
        for (int s = threadIdx.x; s < H; s += blockDim.x) {
            keys[s] = kEmpty;
            kfirst[s] = 0x7fffffff;
            klast[s] = -1;
            kcount[s] = 0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += blockDim.x) {
            const int64_t q = idx[c0 + t];
            if (!on_grid(q)) continue;
            uint32_t h = inject_slot((uint64_t)q, mask);
            for (int probe = 0; probe < H; ++probe) {  // H >= 2 cn: a free slot exists
                const unsigned long long prev = atomicCAS(&keys[h], kEmpty, (unsigned long long)q);
                if (prev == kEmpty || prev == (unsigned long long)q) {
                    atomicMin(&kfirst[h], c0 + t);
                    atomicMax(&klast[h], c0 + t);
                    atomicAdd(&kcount[h], 1);
                    break;
                }
                h = (h + 1) & mask;
            }
        }
        __syncthreads();
        if (!owner) continue;
        uint32_t h = inject_slot((uint64_t)p, mask);
        for (int probe = 0; probe < H; ++probe) {
            const unsigned long long kq = keys[h];
            if (kq == kEmpty) break;  // p does not occur in this chunk
            if (kq == (unsigned long long)p) {
                const int f = kfirst[h], l = klast[h], c = kcount[h];
                if (f < j) {
                    owner = false;  // an earlier source holds this point
                } else if (c <= 2) {
                    v = __builtin_fmaf(kp, row[f] * scale, v);
                    if (l != f) v = __builtin_fmaf(kp, row[l] * scale, v);
                } else {
                    for (int k = f; k <= l; ++k)
                        if (idx[k] == p) v = __builtin_fmaf(kp, row[k] * scale, v);
                }
                break;
            }
            h = (h + 1) & mask;
        }
    }
    if (owner) u[p] = (ST)v;
}

// FP32 field <-> storage: to storage dst = round(src * scale) (nearest even),
// back dst = src / scale (scale is a power of two, so both scalings are exact).
template <typename ST>
__global__ void __launch_bounds__(256) convert_kernel(const void *src, void *dst, int64_t n, float scale,
                                                      int to_storage)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float inv = 1.0f / scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (to_storage)
            ((ST *)dst)[i] = (ST)(((const float *)src)[i] * scale);
        else
            ((float *)dst)[i] = (float)((const ST *)src)[i] * inv;
    }
}

// Receiver samples: out[j] = u[idx[j]] (0 for an index outside the grid).
__global__ void __launch_bounds__(256) sample_kernel(const float *u, int64_t n_points, int64_t pitch, int64_t nx,
                                                     const int64_t *idx, int n, float *out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t p = idx[j];
    out[j] = (p >= 0 && p < n_points && (pitch == nx || p % pitch < nx)) ? u[p] : 0.0f;
}

// Gradient accumulation (FP64): g += s * mu * (u^{k} - 2 u^{k-1} + u^{k-2}).
__global__ void __launch_bounds__(256) grad_kernel(double *g, const float *mu, const float *un, const float *uc,
                                                   const float *up, int64_t n, double s)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double d2 = ((double)un[i] - 2.0 * (double)uc[i]) + (double)up[i];
        g[i] += s * ((double)mu[i] * d2);
    }
}

// Same, four points per thread from 16-byte FP32 vectors and two 16-byte FP64
// pairs, each workgroup streaming one contiguous chunk (n4 = points / 4).
constexpr int64_t kGradChunk = 1024;  // float4 groups per workgroup

__global__ void __launch_bounds__(256) grad_kernel_vec4(double *g, const float *mu, const float *un, const float *uc,
                                                        const float *up, int64_t n4, double s)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef double d2v __attribute__((ext_vector_type(2)));
    const int64_t beg = (int64_t)blockIdx.x * kGradChunk;
    const int64_t end = (beg + kGradChunk < n4) ? beg + kGradChunk : n4;
    for (int64_t i = beg + threadIdx.x; i < end; i += 256) {
        const f4v m = __builtin_nontemporal_load((const f4v *)mu + i);
        const f4v a = __builtin_nontemporal_load((const f4v *)un + i);
        const f4v b = __builtin_nontemporal_load((const f4v *)uc + i);
        const f4v c = __builtin_nontemporal_load((const f4v *)up + i);
        d2v *gp = (d2v *)g + 2 * i;
        d2v g0 = gp[0], g1 = gp[1];
        g0.x += s * ((double)m.x * (((double)a.x - 2.0 * (double)b.x) + (double)c.x));
        g0.y += s * ((double)m.y * (((double)a.y - 2.0 * (double)b.y) + (double)c.y));
        g1.x += s * ((double)m.z * (((double)a.z - 2.0 * (double)b.z) + (double)c.z));
        g1.y += s * ((double)m.w * (((double)a.w - 2.0 * (double)b.w) + (double)c.w));
        gp[0] = g0;
        gp[1] = g1;
    }
}

// M consecutive gradient terms in one pass (adjoint steps k, k-1, ..., k-M+1):
// g = (((g + t_0) + t_1) + ...) with t_j = s mu_j ((u_j - 2 u_{j+1}) + u_{j+2}),
// each term rounded and added exactly as the single-term kernel does, so the
// result is the bits of M single-term passes. Per point: (2M + 2) FP32 reads
// and one FP64 read-modify-write (for M = 4: 56 B instead of 4 x 32 B).
constexpr int kMaxTerms = 4;
struct GradTerms {
    const float *mu[kMaxTerms];
    const float *u[kMaxTerms + 2];
};

template <int M>
__global__ void __launch_bounds__(256) gradn_kernel(double *g, GradTerms f, int64_t n, double s)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double u[M + 2];
#pragma unroll
        for (int j = 0; j < M + 2; ++j) u[j] = (double)f.u[j][i];
        double r = g[i];
#pragma unroll
        for (int j = 0; j < M; ++j) r = r + s * ((double)f.mu[j][i] * ((u[j] - 2.0 * u[j + 1]) + u[j + 2]));
        g[i] = r;
    }
}

template <int M>
__global__ void __launch_bounds__(256) gradn_kernel_vec4(double *g, GradTerms f, int64_t n4, double s)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef double d2v __attribute__((ext_vector_type(2)));
    const int64_t beg = (int64_t)blockIdx.x * kGradChunk;
    const int64_t end = (beg + kGradChunk < n4) ? beg + kGradChunk : n4;
    for (int64_t i = beg + threadIdx.x; i < end; i += 256) {
        f4v m[M], v[M + 2];
#pragma unroll
        for (int j = 0; j < M; ++j) m[j] = __builtin_nontemporal_load((const f4v *)f.mu[j] + i);
#pragma unroll
        for (int j = 0; j < M + 2; ++j) v[j] = __builtin_nontemporal_load((const f4v *)f.u[j] + i);
        d2v *gp = (d2v *)g + 2 * i;
        double r[4] = {gp[0].x, gp[0].y, gp[1].x, gp[1].y};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int j = 0; j < M; ++j)
                r[e] = r[e] + s * ((double)m[j][e] *
                                   (((double)v[j][e] - 2.0 * (double)v[j + 1][e]) + (double)v[j + 2][e]));
        gp[0] = d2v{r[0], r[1]};
        gp[1] = d2v{r[2], r[3]};
    }
}

// resid = traces - observed (FP32), misfit = 1/2 sum resid^2 accumulated in
// FP64 by one workgroup in a fixed order (deterministic).
constexpr int kMisfitThreads = 1024;

__global__ void __launch_bounds__(kMisfitThreads) misfit_kernel(const float *tr, const float *obs, int64_t count,
                                                                float *resid, double *misfit)
{
    __shared__ double part[kMisfitThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kMisfitThreads) {
        const float r = tr[i] - obs[i];
        if (resid) resid[i] = r;
        acc += (double)r * (double)r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kMisfitThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *misfit = 0.5 * part[0];
}


// Divergence watchdog: the largest magnitude over n stored values as the
// bit pattern of a non-negative float. For non-negative floats the unsigned
// order of the patterns is the numeric order, NaN patterns lie above +inf,
// so an unsigned maximum gives NaN if any value is NaN, else +inf if any is
// infinite, else max |u|. Each workgroup reduces in LDS and adds one atomic.
__global__ void __launch_bounds__(64) max_abs_clear_kernel(unsigned int *out)
{
    if (threadIdx.x == 0) *out = 0u;
}

template <typename ST>
__global__ void __launch_bounds__(256) max_abs_kernel(const ST *u, int64_t n, unsigned int *out)
{
    __shared__ unsigned int part[256];
    unsigned int m = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        m = max(m, __float_as_uint(fabsf((float)u[i])));
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = max(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, part[0]);
}

__global__ void __launch_bounds__(256) max_abs_kernel_vec4(const float4 *u, int64_t n4, unsigned int *out)
{
    __shared__ unsigned int part[256];
    unsigned int m = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = u[i];
        m = max(m, max(max(__float_as_uint(fabsf(v.x)), __float_as_uint(fabsf(v.y))),
                       max(__float_as_uint(fabsf(v.z)), __float_as_uint(fabsf(v.w)))));
    }
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = max(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, part[0]);
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Streaming reference: out = a (+ b) (+ c), NIN inputs, one output. Each
// workgroup streams one contiguous chunk of kStreamChunk 16-byte vectors,
// four loads per input in flight per thread before the stores, all
// non-temporal (the fastest of the simple streaming patterns measured on
// MI355X). NIN = 1 is a copy; NIN = 3 has the sweep's three reads per write.
constexpr int kStreamUnroll = 4;
constexpr int64_t kStreamChunk = 4096;

template <int NIN>
__global__ void __launch_bounds__(256) stream_kernel(const f4 *a, const f4 *b, const f4 *c, f4 *out, int64_t n4)
{
    const int64_t beg = (int64_t)blockIdx.x * kStreamChunk;
    const int64_t end = (beg + kStreamChunk < n4) ? beg + kStreamChunk : n4;
    int64_t i = beg + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * 256 < end; i += kStreamUnroll * 256) {
        f4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            v[u] = __builtin_nontemporal_load(&a[i + u * 256]);
            if (NIN > 1) v[u] += __builtin_nontemporal_load(&b[i + u * 256]);
            if (NIN > 2) v[u] += __builtin_nontemporal_load(&c[i + u * 256]);
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) __builtin_nontemporal_store(v[u], &out[i + u * 256]);
    }
    for (; i < end; i += 256) {
        f4 v = __builtin_nontemporal_load(&a[i]);
        if (NIN > 1) v += __builtin_nontemporal_load(&b[i]);
        if (NIN > 2) v += __builtin_nontemporal_load(&c[i]);
        __builtin_nontemporal_store(v, &out[i]);
    }
}

// The same three-read, one-write stream in the one-step sweep's access order,
// without the stencil: [nz][ny][nx] FP32 fields (nx % 4 == 0), a workgroup
// of 64 x 4 threads owns a column of 64 four-float vectors x 4 rows and
// marches kMarchDz planes; u^n-like input `a` cached, the others and the
// output non-temporal, as in the sweep.
constexpr int kMarchDz = 256;

__global__ void __launch_bounds__(256) stream_march_kernel(const f4 *a, const f4 *b, const f4 *c, f4 *out, int nxv,
                                                           int ny, int nz, int gx, int gy)
{
    const int blk = blockIdx.x;
    const int x = (blk % gx) * 64 + (int)(threadIdx.x % 64);
    const int y = ((blk / gx) % gy) * 4 + (int)(threadIdx.x / 64);
    const int z0 = (blk / gx / gy) * kMarchDz;
    const int z1 = (z0 + kMarchDz < nz) ? z0 + kMarchDz : nz;
    if (x >= nxv || y >= ny) return;
    const int64_t plane = (int64_t)nxv * ny;
    for (int z = z0; z < z1; ++z) {
        const int64_t i = z * plane + (int64_t)y * nxv + x;
        const f4 v = (a[i] + __builtin_nontemporal_load(&b[i])) + __builtin_nontemporal_load(&c[i]);
        __builtin_nontemporal_store(v, &out[i]);
    }
}

// Same for any size and 4-byte alignment, one float per thread per step.
template <int NIN>
__global__ void __launch_bounds__(256) stream_kernel_scalar(const float *a, const float *b, const float *c, float *out,
                                                            int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float v = __builtin_nontemporal_load(&a[i]);
        if (NIN > 1) v += __builtin_nontemporal_load(&b[i]);
        if (NIN > 2) v += __builtin_nontemporal_load(&c[i]);
        __builtin_nontemporal_store(v, &out[i]);
    }
}

}  // namespace

int zmarch_variant_count() { return registry().n; }

const ZVariant *zmarch_variant(int i)
{
    const Registry &r = registry();
    return (i >= 0 && i < r.n) ? r.items[i] : nullptr;
}

int zmarch2_variant_count() { return registry2().n; }

const Z2Variant *zmarch2_variant(int i)
{
    const Registry2 &r = registry2();
    return (i >= 0 && i < r.n) ? r.items[i] : nullptr;
}

hipError_t launch_zmarch2(const Z2Variant &v, const SweepArgs &a, hipStream_t s)
{
    const int blocks = a.gx * a.gy * a.gz;
    hipLaunchKernelGGL(v.kernel, dim3(blocks), dim3(v.threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zmarch(const ZVariant &v, const SweepArgs &a, hipStream_t s)
{
    const int blocks = a.gx * a.gy * a.gz;
    hipLaunchKernelGGL(v.kernel, dim3(blocks), dim3(v.threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zmarch_batch(const ZVariant &v, const SweepArgs *shots, const int *wg_begin, int nshots,
                               int total_blocks, int xcd, int64_t it, hipStream_t s)
{
    hipLaunchKernelGGL(v.batch_kernel, dim3(total_blocks), dim3(v.threads), 0, s, shots, wg_begin, nshots, xcd, it);
    return hipGetLastError();
}

hipError_t launch_plain(int R, int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s)
{
    switch (R) {
    case 3: return launch_plain_r3(st, bx, by, bz, a, s);
    case 4: return launch_plain_r4(st, bx, by, bz, a, s);
    case 5: return launch_plain_r5(st, bx, by, bz, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inject(int st, void *u, const float *kappa, int64_t n_points, int64_t pitch, int64_t nx,
                         const int64_t *idx, const float *amp, int nsrc, int64_t it, float scale, hipStream_t s)
{
    const dim3 grid((nsrc + 255) / 256), block(256);
    switch (st) {
    case kF32:
        hipLaunchKernelGGL(inject_kernel<float>, grid, block, 0, s, (float *)u, kappa, n_points, pitch, nx, idx, amp,
                           nsrc, it, scale);
        break;
    case kF16:
        hipLaunchKernelGGL(inject_kernel<_Float16>, grid, block, 0, s, (_Float16 *)u, kappa, n_points, pitch, nx, idx,
                           amp, nsrc, it, scale);
        break;
    case kBF16:
        hipLaunchKernelGGL(inject_kernel<__bf16>, grid, block, 0, s, (__bf16 *)u, kappa, n_points, pitch, nx, idx, amp,
                           nsrc, it, scale);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int st, const void *src, void *dst, int64_t n, float scale, int to_storage, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    switch (st) {
    case kF32:
        hipLaunchKernelGGL(convert_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, scale,
                           to_storage);
        break;
    case kF16:
        hipLaunchKernelGGL(convert_kernel<_Float16>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, scale,
                           to_storage);
        break;
    case kBF16:
        hipLaunchKernelGGL(convert_kernel<__bf16>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, scale,
                           to_storage);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kappa_m(const float *m, float *kappa, int64_t n, double dt, double h, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kappa_m_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, kappa, n, dt, h);
    return hipGetLastError();
}

hipError_t launch_sample(const float *u, int64_t n_points, int64_t pitch, int64_t nx, const int64_t *idx, int n,
                         float *out, hipStream_t s)
{
    hipLaunchKernelGGL(sample_kernel, dim3((n + 255) / 256), dim3(256), 0, s, u, n_points, pitch, nx, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_grad(double *g, const float *mu, const float *un, const float *uc, const float *up, int64_t n,
                       double scale, hipStream_t s)
{
    if (n % 4 == 0 && !(((uintptr_t)g | (uintptr_t)mu | (uintptr_t)un | (uintptr_t)uc | (uintptr_t)up) & 15u)) {
        const int64_t n4 = n / 4;
        const int64_t blocks = (n4 + kGradChunk - 1) / kGradChunk;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(grad_kernel_vec4, dim3((unsigned)blocks), dim3(256), 0, s, g, mu, un, uc, up, n4, scale);
        return hipGetLastError();
    }
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(grad_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, mu, un, uc, up, n, scale);
    return hipGetLastError();
}

hipError_t launch_gradn(int m, double *g, const float *const *mu, const float *const *u, int64_t n, double scale,
                        hipStream_t s)
{
    if (m < 1 || m > kMaxTerms) return hipErrorInvalidValue;
    GradTerms f = {};
    uintptr_t bits = (uintptr_t)g;
    for (int j = 0; j < m; ++j) {
        f.mu[j] = mu[j];
        bits |= (uintptr_t)mu[j];
    }
    for (int j = 0; j < m + 2; ++j) {
        f.u[j] = u[j];
        bits |= (uintptr_t)u[j];
    }
    if (n % 4 == 0 && !(bits & 15u)) {
        const int64_t n4 = n / 4;
        const int64_t blocks = (n4 + kGradChunk - 1) / kGradChunk;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        const dim3 grid((unsigned)blocks), block(256);
        switch (m) {
        case 1: hipLaunchKernelGGL(gradn_kernel_vec4<1>, grid, block, 0, s, g, f, n4, scale); break;
        case 2: hipLaunchKernelGGL(gradn_kernel_vec4<2>, grid, block, 0, s, g, f, n4, scale); break;
        case 3: hipLaunchKernelGGL(gradn_kernel_vec4<3>, grid, block, 0, s, g, f, n4, scale); break;
        default: hipLaunchKernelGGL(gradn_kernel_vec4<4>, grid, block, 0, s, g, f, n4, scale); break;
        }
        return hipGetLastError();
    }
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks), block(256);
    switch (m) {
    case 1: hipLaunchKernelGGL(gradn_kernel<1>, grid, block, 0, s, g, f, n, scale); break;
    case 2: hipLaunchKernelGGL(gradn_kernel<2>, grid, block, 0, s, g, f, n, scale); break;
    case 3: hipLaunchKernelGGL(gradn_kernel<3>, grid, block, 0, s, g, f, n, scale); break;
    default: hipLaunchKernelGGL(gradn_kernel<4>, grid, block, 0, s, g, f, n, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_misfit(const float *tr, const float *obs, int64_t count, float *resid, double *misfit, hipStream_t s)
{
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(kMisfitThreads), 0, s, tr, obs, count, resid, misfit);
    return hipGetLastError();
}

hipError_t launch_kappa(const float *v, float *kappa, int64_t n, double dt, double h, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kappa_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v, kappa, n, dt, h);
    return hipGetLastError();
}

hipError_t launch_max_abs(int st, const void *u, int64_t n, unsigned int *out, hipStream_t s)
{
    hipLaunchKernelGGL(max_abs_clear_kernel, dim3(1), dim3(64), 0, s, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n + 1023) / 1024, 1), 4096);
    switch (st) {
    case kF32:
        if (n % 4 == 0 && !((uintptr_t)u & 15u))
            hipLaunchKernelGGL(max_abs_kernel_vec4, dim3((unsigned)blocks), dim3(256), 0, s, (const float4 *)u, n / 4,
                               out);
        else
            hipLaunchKernelGGL(max_abs_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float *)u, n, out);
        break;
    case kF16:
        hipLaunchKernelGGL(max_abs_kernel<_Float16>, dim3((unsigned)blocks), dim3(256), 0, s, (const _Float16 *)u, n,
                           out);
        break;
    case kBF16:
        hipLaunchKernelGGL(max_abs_kernel<__bf16>, dim3((unsigned)blocks), dim3(256), 0, s, (const __bf16 *)u, n, out);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stream_march(const void *a, const void *b, const void *c, void *out, int64_t nx, int64_t ny,
                              int64_t nz, hipStream_t s)
{
    const int nxv = (int)(nx / 4);
    const int64_t gx = (nxv + 63) / 64, gy = (ny + 3) / 4, gz = (nz + kMarchDz - 1) / kMarchDz;
    if (gx * gy * gz > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_march_kernel, dim3((unsigned)(gx * gy * gz)), dim3(256), 0, s, (const f4 *)a,
                       (const f4 *)b, (const f4 *)c, (f4 *)out, nxv, (int)ny, (int)nz, (int)gx, (int)gy);
    return hipGetLastError();
}

hipError_t launch_stream(const void *a, const void *b, const void *c, void *out, int64_t nbytes, hipStream_t s)
{
    if ((nbytes % 16) || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)out) & 15u)) {
        const int64_t n = nbytes / 4;
        int64_t blocks = (n + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        const float *sa = (const float *)a, *sb = (const float *)b, *sc = (const float *)c;
        if (c)
            hipLaunchKernelGGL(stream_kernel_scalar<3>, dim3((unsigned)blocks), dim3(256), 0, s, sa, sb, sc,
                               (float *)out, n);
        else if (b)
            hipLaunchKernelGGL(stream_kernel_scalar<2>, dim3((unsigned)blocks), dim3(256), 0, s, sa, sb, sc,
                               (float *)out, n);
        else
            hipLaunchKernelGGL(stream_kernel_scalar<1>, dim3((unsigned)blocks), dim3(256), 0, s, sa, sb, sc,
                               (float *)out, n);
        return hipGetLastError();
    }
    const int64_t n4 = nbytes / 16;
    const int64_t blocks = (n4 + kStreamChunk - 1) / kStreamChunk;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const f4 *fa = (const f4 *)a, *fb = (const f4 *)b, *fc = (const f4 *)c;
    if (c)
        hipLaunchKernelGGL(stream_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, fa, fb, fc, (f4 *)out, n4);
    else if (b)
        hipLaunchKernelGGL(stream_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, fa, fb, fc, (f4 *)out, n4);
    else
        hipLaunchKernelGGL(stream_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, fa, fb, fc, (f4 *)out, n4);
    return hipGetLastError();
}

}  // namespace p1310
