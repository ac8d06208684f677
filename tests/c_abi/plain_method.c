/* A C program that drives the library through the C ABI alone (no Python, no
 * torch): the plain-method workload (constant velocity, centred point source,
 * zero ghost layer) on an nx x ny x nz grid for nt steps, 8th order.
 *
 *   plain_method <nx> <ny> <nz> <nt> <wavelet.f32> <out.f32>
 *
 * wavelet.f32 holds nt FP32 source samples; out.f32 receives u^nt then
 * u^{nt-1} (FP32, [nz][ny][nx] each). Exit status 0 on success. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "../../include/stencil.h"

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 2;                                                         \
        }                                                                     \
    } while (0)

static int check(stencil_status st, const stencil_ctx *ctx, const char *what)
{
    if (st == STENCIL_OK) return 0;
    fprintf(stderr, "%s: %s (%s)\n", what, stencil_strerror(st), stencil_last_error(ctx));
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: %s nx ny nz nt wavelet.f32 out.f32\n", argv[0]);
        return 2;
    }
    const int64_t nx = atoll(argv[1]), ny = atoll(argv[2]), nz = atoll(argv[3]);
    const int64_t nt = atoll(argv[4]);
    const int64_t n = nx * ny * nz;
    const double h = 10.0, vel = 2000.0, dt = 0.4 * h / vel;

    float *w = (float *)malloc((size_t)nt * sizeof(float));
    float *host = (float *)malloc((size_t)n * sizeof(float));
    if (!w || !host) return 2;
    FILE *f = fopen(argv[5], "rb");
    if (!f || fread(w, sizeof(float), (size_t)nt, f) != (size_t)nt) {
        fprintf(stderr, "cannot read %lld wavelet samples from %s\n", (long long)nt, argv[5]);
        return 2;
    }
    fclose(f);
    for (int64_t i = 0; i < n; ++i) host[i] = (float)vel;

    float *v, *kappa, *a, *b, *amp;
    int64_t *idx;
    HIP_OK(hipMalloc((void **)&v, n * sizeof(float)));
    HIP_OK(hipMalloc((void **)&kappa, n * sizeof(float)));
    HIP_OK(hipMalloc((void **)&a, n * sizeof(float)));
    HIP_OK(hipMalloc((void **)&b, n * sizeof(float)));
    HIP_OK(hipMalloc((void **)&amp, nt * sizeof(float)));
    HIP_OK(hipMalloc((void **)&idx, sizeof(int64_t)));
    HIP_OK(hipMemcpy(v, host, n * sizeof(float), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(amp, w, nt * sizeof(float), hipMemcpyHostToDevice));
    const int64_t s = ((nz / 2) * ny + ny / 2) * nx + nx / 2;
    HIP_OK(hipMemcpy(idx, &s, sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemset(a, 0, n * sizeof(float)));
    HIP_OK(hipMemset(b, 0, n * sizeof(float)));

    stencil_desc d = {0};
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.radius = 4;
    d.storage = STENCIL_F32;
    d.h = h;
    d.dt = dt;
    d.vmax = vel;
    d.device = 0;
    d.storage_scale = 1.0;
    stencil_ctx *ctx = NULL;
    if (check(stencil_init(&d, &ctx), NULL, "stencil_init")) return 1;
    if (check(stencil_kappa(ctx, v, kappa, NULL), ctx, "stencil_kappa")) return 1;
    stencil_src src = {1, idx, amp, nt};
    for (int64_t it = 0; it < nt; ++it) {
        if (check(stencil_step(ctx, kappa, a, b, it, &src, NULL), ctx, "stencil_step")) return 1;
        float *t = a;  /* b now holds u^{it+1} */
        a = b;
        b = t;
    }
    HIP_OK(hipDeviceSynchronize());
    f = fopen(argv[6], "wb");
    if (!f) return 2;
    HIP_OK(hipMemcpy(host, a, n * sizeof(float), hipMemcpyDeviceToHost));
    fwrite(host, sizeof(float), (size_t)n, f);
    HIP_OK(hipMemcpy(host, b, n * sizeof(float), hipMemcpyDeviceToHost));
    fwrite(host, sizeof(float), (size_t)n, f);
    fclose(f);
    stencil_tile t;
    stencil_get_tile(ctx, &t);
    printf("plain_method: %lldx%lldx%lld, %lld steps, tile kind %d %dx%d ry %d vw %d dz %d\n", (long long)nx,
           (long long)ny, (long long)nz, (long long)nt, t.kind, t.bx, t.by, t.ry, t.vw, t.dz);
    stencil_destroy(ctx);
    hipFree(v);
    hipFree(kappa);
    hipFree(a);
    hipFree(b);
    hipFree(amp);
    hipFree(idx);
    free(w);
    free(host);
    return 0;
}
