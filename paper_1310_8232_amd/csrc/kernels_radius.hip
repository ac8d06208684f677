// Instantiations of the sweep kernels for one radius (RADIUS is set on the
// compiler command line; the library links one object per radius).
#include "sweep.hpp"

#ifndef RADIUS
#error "compile with -DRADIUS=<3|4|5>"
#endif

namespace p1310 {

#define P1310_CAT2(a, b) a##b
#define P1310_CAT(a, b) P1310_CAT2(a, b)

// (BX, BY, RY, VW, PF) of every z-march instantiation.
#define ZV(BX, BY, RY, VW, PF)                                                                  \
    {RADIUS, BX, BY, RY, VW, PF, zmarch_kernel<RADIUS, BX, BY, RY, VW, PF>,                     \
     zmarch_batch_kernel<RADIUS, BX, BY, RY, VW, PF>, BX * BY,                                  \
     (int)(2 * (((BY * RY + 2 * RADIUS) * (BX * VW + 2 * ((VW == 1) ? RADIUS : ((RADIUS + VW - 1) / VW) * VW))) + VW) * 4)},

static const ZVariant kTable[] = {
    ZV(16, 4, 1, 4, 0) ZV(16, 4, 2, 4, 0)
    ZV(16, 8, 1, 4, 0) ZV(16, 8, 2, 4, 0)
    ZV(16, 16, 1, 4, 0) ZV(16, 16, 2, 4, 0)
    ZV(32, 4, 1, 4, 0) ZV(32, 4, 2, 4, 0)
    ZV(32, 8, 1, 4, 0) ZV(32, 8, 2, 4, 0)
    ZV(64, 2, 2, 4, 0) ZV(64, 4, 1, 4, 0) ZV(64, 4, 2, 4, 0)
    ZV(64, 2, 1, 4, 0) ZV(64, 8, 1, 4, 0) ZV(32, 16, 1, 4, 0) ZV(128, 2, 1, 4, 0) ZV(128, 4, 1, 4, 0)
    ZV(64, 8, 1, 4, 1) ZV(128, 2, 1, 4, 1)
    ZV(16, 4, 2, 4, 1) ZV(16, 8, 1, 4, 1) ZV(16, 8, 2, 4, 1) ZV(16, 16, 1, 4, 1)
    ZV(32, 4, 2, 4, 1) ZV(32, 8, 1, 4, 1) ZV(64, 4, 1, 4, 1)
    ZV(64, 4, 1, 1, 0) ZV(64, 4, 2, 1, 0) ZV(32, 8, 2, 1, 0) ZV(64, 8, 1, 1, 0)
};

const ZVariant *P1310_CAT(zmarch_table_r, RADIUS)(int *n)
{
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

hipError_t P1310_CAT(launch_plain_r, RADIUS)(int bx, int by, int bz, const SweepArgs &a, hipStream_t s)
{
    dim3 block(bx, by, bz);
    dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, (a.nz + bz - 1) / bz);
    hipLaunchKernelGGL(plain_kernel<RADIUS>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace p1310
