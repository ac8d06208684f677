// Internal interface between the C-ABI runtime (api.cpp) and the gfx950
// kernels (kernels.hip). Not installed; the public interface is
// include/stencil.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p1310 {

constexpr int kMaxRadius = 5;

// Arguments of one sweep launch (passed by value as the kernel argument).
struct SweepArgs {
    const float *kappa;      // [nz][ny][nx], FP32
    const void *ucur;        // u^n (storage type of the variant)
    const void *uprev;       // u^{n-1}
    void *unext;             // u^{n+1} (may be uprev: in-place update)
    void *unext2;            // u^{n+2} (two-step kernels only)
    int nx, ny, nz;
    int pitch;               // row stride in values (>= nx); point (z,y,x) at (z*ny + y)*pitch + x
    int dz;                  // planes per workgroup (z-march)
    int gx, gy, gz;          // tiles along x, y and z-chunks
    int xcd;                 // 0 = linear workgroup order, else number of XCDs to spread over
    float c[kMaxRadius + 1]; // c[0] = 3*c_0, c[m] = c_m
    const int64_t *src_idx;  // fused single source (nsrc == 1), else unused
    const float *src_amp;
    int nsrc;
    int64_t it;
    float scale;             // storage scale: source amplitudes are multiplied by it
    int pace;                // two-step kernels: edge pacing code 0..7 (0 = off)
};

// Wavefield storage types (stencil_storage).
constexpr int kF32 = 0, kF16 = 1, kBF16 = 2;

// One compiled z-march instantiation.
struct ZVariant {
    int R, bx, by, ry, vw, pf, st;
    void (*kernel)(SweepArgs);
    void (*batch_kernel)(const SweepArgs *, const int *, int, int, int64_t);
    int threads;
    int lds_bytes;
};

// Registry of compiled z-march kernels (kernels.hip).
int zmarch_variant_count();
const ZVariant *zmarch_variant(int i);

// One compiled two-step (temporally blocked) z-march instantiation: a
// workgroup of bx x by threads covers an extended tile of (bx*vw) x by points,
// its own tile is (bx*vw - 2*hx) x (by - 2R).
struct Z2Variant {
    int R, bx, by, vw, pf, st;
    void (*kernel)(SweepArgs);
    int threads;
    int own_x, own_y;
};
int zmarch2_variant_count();
const Z2Variant *zmarch2_variant(int i);
hipError_t launch_zmarch2(const Z2Variant &v, const SweepArgs &a, hipStream_t s);

// Launchers (kernels.hip). All enqueue on `s` and return the launch status.
hipError_t launch_zmarch(const ZVariant &v, const SweepArgs &a, hipStream_t s);
hipError_t launch_zmarch_batch(const ZVariant &v, const SweepArgs *shots, const int *wg_begin, int nshots,
                               int total_blocks, int xcd, int64_t it, hipStream_t s);
hipError_t launch_plain(int R, int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s);
// Sources whose index is outside [0, n_points) or falls in a row's padding
// (index mod pitch >= nx) are skipped.
hipError_t launch_inject(int st, void *u, const float *kappa, int64_t n_points, int64_t pitch, int64_t nx,
                         const int64_t *idx, const float *amp, int nsrc, int64_t it, float scale, hipStream_t s);
hipError_t launch_convert(int st, const void *src, void *dst, int64_t n, float scale, int to_storage,
                          hipStream_t s);
hipError_t launch_kappa(const float *v, float *kappa, int64_t n, double dt, double h, hipStream_t s);
hipError_t launch_kappa_m(const float *m, float *kappa, int64_t n, double dt, double h, hipStream_t s);
hipError_t launch_sample(const float *u, int64_t n_points, int64_t pitch, int64_t nx, const int64_t *idx, int n,
                         float *out, hipStream_t s);
hipError_t launch_grad(double *g, const float *mu, const float *un, const float *uc, const float *up, int64_t n,
                       double scale, hipStream_t s);
// m = 1..4 consecutive gradient terms: mu[0..m-1], u[0..m+1] (see gradn_kernel).
hipError_t launch_gradn(int m, double *g, const float *const *mu, const float *const *u, int64_t n, double scale,
                        hipStream_t s);
hipError_t launch_misfit(const float *tr, const float *obs, int64_t count, float *resid, double *misfit,
                         hipStream_t s);
// Largest |u| (bit pattern, NaN above +inf above finite) of n stored values into *out.
hipError_t launch_max_abs(int st, const void *u, int64_t n, unsigned int *out, hipStream_t s);
hipError_t launch_stream_march(const void *a, const void *b, const void *c, void *out, int64_t nx, int64_t ny,
                              int64_t nz, hipStream_t s);
hipError_t launch_stream(const void *a, const void *b, const void *c, void *out, int64_t nbytes, hipStream_t s);

}  // namespace p1310
