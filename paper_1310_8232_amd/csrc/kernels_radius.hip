// Instantiations of the sweep kernels for one radius (RADIUS is set on the
// compiler command line; the library links one object per radius).
#include "sweep.hpp"
#include "sweep2.hpp"
#include "sweep_batch.hpp"

#ifndef RADIUS
#error "compile with -DRADIUS=<3|4|5>"
#endif

namespace p1310 {

#define P1310_CAT2(a, b) a##b
#define P1310_CAT(a, b) P1310_CAT2(a, b)

// Storage type tags of the table (kF32 / kF16 / kBF16) and their C++ types.
#define ST_kF32 float
#define ST_kF16 _Float16
#define ST_kBF16 __bf16

// LDS bytes of a (BX, BY, RY, VW) tile: two planes of (TY + 2R) x (TX + 2HX) FP32 values.
#define ZV_LDS(BX, BY, RY, VW)                                                                   \
    (int)(2 * (((BY * RY + 2 * RADIUS) * (BX * VW + 2 * ((VW == 1) ? RADIUS : ((RADIUS + VW - 1) / VW) * VW))) + VW) * 4)

// One z-march instantiation: (BX, BY, RY, VW, PF) and the storage tag.
#define ZVS(BX, BY, RY, VW, PF, STT)                                                             \
    {RADIUS, BX, BY, RY, VW, PF, STT, zmarch_kernel<RADIUS, BX, BY, RY, VW, PF, ST_##STT>,       \
     zmarch_batch_kernel<RADIUS, BX, BY, RY, VW, PF, ST_##STT>, BX * BY, ZV_LDS(BX, BY, RY, VW)},
#define ZV(BX, BY, RY, VW, PF) ZVS(BX, BY, RY, VW, PF, kF32)

// 16-bit wavefield storage (radii 4 and 5): four- and eight-point vectors (an
// eight-point vector of 16-bit values is one 16-byte access), one-point rows,
// and tiles of 16 and 32 rows (less y halo per point).
#if RADIUS >= 4
// Eight-point tiles of four rows, and the prefetching eight-point tile, spill
// registers at R = 5 (4-6 VGPRs); they are compiled for R = 4 only.
#if RADIUS == 4
#define ZV16_R4ONLY(STT) ZVS(32, 4, 1, 8, 0, STT) ZVS(64, 4, 1, 8, 0, STT) ZVS(32, 8, 1, 8, 1, STT)
#else
#define ZV16_R4ONLY(STT)
#endif
#define ZV16(STT)                                                                                \
    ZVS(16, 8, 1, 4, 0, STT) ZVS(16, 8, 2, 4, 0, STT) ZVS(32, 8, 1, 4, 0, STT)                  \
    ZVS(32, 4, 2, 4, 0, STT) ZVS(64, 4, 1, 4, 0, STT) ZVS(64, 4, 2, 4, 0, STT)                  \
    ZVS(16, 16, 1, 4, 0, STT) ZVS(64, 4, 1, 4, 1, STT) ZVS(64, 4, 1, 1, 0, STT)                  \
    ZVS(128, 2, 1, 4, 0, STT) ZVS(32, 16, 1, 4, 0, STT) ZVS(64, 8, 1, 4, 0, STT)                 \
    ZVS(16, 8, 1, 8, 0, STT) ZVS(32, 8, 1, 8, 0, STT) ZVS(16, 16, 1, 8, 0, STT)                  \
    ZVS(32, 16, 2, 4, 0, STT) ZVS(16, 16, 2, 4, 0, STT) ZVS(32, 8, 2, 4, 0, STT)                 \
    ZVS(64, 8, 2, 4, 0, STT) ZV16_R4ONLY(STT)
#else
#define ZV16(STT)
#endif

static const ZVariant kTable[] = {
    ZV(16, 4, 1, 4, 0) ZV(16, 4, 2, 4, 0)
    ZV(16, 8, 1, 4, 0) ZV(16, 8, 2, 4, 0)
    ZV(16, 16, 1, 4, 0) ZV(16, 16, 2, 4, 0)
    ZV(32, 4, 1, 4, 0) ZV(32, 4, 2, 4, 0)
    ZV(32, 8, 1, 4, 0) ZV(32, 8, 2, 4, 0)
    ZV(64, 2, 2, 4, 0) ZV(64, 4, 1, 4, 0) ZV(64, 4, 2, 4, 0)
    ZV(64, 2, 1, 4, 0) ZV(64, 8, 1, 4, 0) ZV(32, 16, 1, 4, 0) ZV(128, 2, 1, 4, 0) ZV(128, 4, 1, 4, 0)
    ZV(32, 16, 2, 4, 0) ZV(64, 8, 2, 4, 0)
    ZV(64, 8, 1, 4, 1) ZV(128, 2, 1, 4, 1)
    ZV(16, 4, 2, 4, 1) ZV(16, 8, 1, 4, 1) ZV(16, 8, 2, 4, 1) ZV(16, 16, 1, 4, 1)
    ZV(32, 4, 2, 4, 1) ZV(32, 8, 1, 4, 1) ZV(64, 4, 1, 4, 1)
    ZV(64, 4, 1, 1, 0) ZV(64, 4, 2, 1, 0) ZV(32, 8, 2, 1, 0) ZV(64, 8, 1, 1, 0)
    ZV(128, 4, 1, 1, 0) ZV(128, 2, 2, 1, 0) ZV(256, 2, 1, 1, 0)
    ZV(64, 4, 1, 2, 0) ZV(64, 4, 2, 2, 0) ZV(64, 8, 1, 2, 0) ZV(32, 8, 1, 2, 0) ZV(32, 8, 2, 2, 0)
    ZV(128, 2, 1, 2, 0) ZV(128, 4, 1, 2, 0) ZV(64, 4, 1, 2, 1) ZV(128, 2, 1, 2, 1)
    ZV16(kF16) ZV16(kBF16)
};

// Two-step kernels (RY = 1, FP32 storage): (BX, BY, VW, PF). The 8 x 64
// tile with prefetch is not compiled: a branch-free build of the two-step
// kernel gave run-to-run differing values on it and no cause was shown.
#define Z2V(BX, BY, VW, PF)                                                                       \
    {RADIUS, BX, BY, VW, PF, kF32, zmarch2_kernel<RADIUS, BX, BY, VW, PF, float>, BX * BY,       \
     BX * VW - 2 * ((VW == 1) ? RADIUS : ((RADIUS + VW - 1) / VW) * VW), BY - 2 * RADIUS},

// The 18-thread-wide tiles (720 and 576 threads, at most 168 VGPRs per lane)
// spill at R = 5 and are compiled for R = 3, 4 only.
#if RADIUS <= 4
#define Z2V_WIDE Z2V(18, 40, 4, 0) Z2V(18, 32, 4, 0)
#else
#define Z2V_WIDE
#endif

static const Z2Variant kTable2[] = {
    Z2V(16, 32, 4, 0) Z2V(16, 32, 4, 1) Z2V_WIDE Z2V(16, 24, 4, 0)
    Z2V(32, 16, 1, 0)
};

const Z2Variant *P1310_CAT(zmarch2_table_r, RADIUS)(int *n)
{
    *n = (int)(sizeof(kTable2) / sizeof(kTable2[0]));
    return kTable2;
}

const ZVariant *P1310_CAT(zmarch_table_r, RADIUS)(int *n)
{
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

hipError_t P1310_CAT(launch_plain_r, RADIUS)(int st, int bx, int by, int bz, const SweepArgs &a, hipStream_t s)
{
    dim3 block(bx, by, bz);
    dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, (a.nz + bz - 1) / bz);
    switch (st) {
    case kF32: hipLaunchKernelGGL((plain_kernel<RADIUS, float>), grid, block, 0, s, a); break;
#if RADIUS >= 4
    case kF16: hipLaunchKernelGGL((plain_kernel<RADIUS, _Float16>), grid, block, 0, s, a); break;
    case kBF16: hipLaunchKernelGGL((plain_kernel<RADIUS, __bf16>), grid, block, 0, s, a); break;
#endif
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace p1310
