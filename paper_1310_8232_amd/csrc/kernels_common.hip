// Radius-independent kernels (model set-up, multi-source injection, streaming
// bandwidth reference) and the registry/launchers over the per-radius objects.
#include "internal.h"

namespace p1310 {

const ZVariant *zmarch_table_r3(int *n);
const ZVariant *zmarch_table_r4(int *n);
const ZVariant *zmarch_table_r5(int *n);
hipError_t launch_plain_r3(int bx, int by, int bz, const SweepArgs &a, hipStream_t s);
hipError_t launch_plain_r4(int bx, int by, int bz, const SweepArgs &a, hipStream_t s);
hipError_t launch_plain_r5(int bx, int by, int bz, const SweepArgs &a, hipStream_t s);

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

// kappa = (v dt / h)^2 formed in FP64, rounded once to FP32.
__global__ void __launch_bounds__(256) kappa_kernel(const float *v, float *kappa, int64_t n, double dt, double h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double r = (double)v[i] * dt / h;
        kappa[i] = (float)(r * r);
    }
}

// Several point sources, added one after another in index order (so that
// repeated indices accumulate deterministically).
__global__ void __launch_bounds__(64) inject_kernel(float *u, const float *kappa, int64_t n_points,
                                                    const int64_t *idx, const float *amp, int nsrc, int64_t it)
{
    if (threadIdx.x != 0) return;
    for (int j = 0; j < nsrc; ++j) {
        const int64_t p = idx[j];
        if (p < 0 || p >= n_points) continue;
        u[p] = __builtin_fmaf(kappa[p], amp[it * nsrc + j], u[p]);
    }
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

}  // namespace

int zmarch_variant_count() { return registry().n; }

const ZVariant *zmarch_variant(int i)
{
    const Registry &r = registry();
    return (i >= 0 && i < r.n) ? r.items[i] : nullptr;
}

hipError_t launch_zmarch(const ZVariant &v, const SweepArgs &a, hipStream_t s)
{
    const int blocks = a.gx * a.gy * a.gz;
    hipLaunchKernelGGL(v.kernel, dim3(blocks), dim3(v.threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_plain(int R, int bx, int by, int bz, const SweepArgs &a, hipStream_t s)
{
    switch (R) {
    case 3: return launch_plain_r3(bx, by, bz, a, s);
    case 4: return launch_plain_r4(bx, by, bz, a, s);
    case 5: return launch_plain_r5(bx, by, bz, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inject(float *u, const float *kappa, int64_t n_points, const int64_t *idx,
                         const float *amp, int nsrc, int64_t it, hipStream_t s)
{
    hipLaunchKernelGGL(inject_kernel, dim3(1), dim3(64), 0, s, u, kappa, n_points, idx, amp, nsrc, it);
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

hipError_t launch_stream(const void *a, const void *b, const void *c, void *out, int64_t nbytes, hipStream_t s)
{
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
