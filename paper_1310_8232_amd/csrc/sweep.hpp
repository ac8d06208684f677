// gfx950 kernels of the leapfrog star-stencil step (paper: Section 2, the
// "3D model" step of Algorithm 1; star stencil of Fig. 1(a); loop blocking of
// Section 3 / Fig. 1(b)).
//
// Per point p (canonical FP32 operation order, shared by every kernel so that
// every tile shape gives bit-identical results):
//   acc = (3 c_0) u(p)
//   for m = 1..R:  s_m = ((x+ + x-) + (y+ + y-)) + (z+ + z-);  acc = fma(c_m, s_m, acc)
//   u^{n+1}(p) = fma(kappa(p), acc, fma(2, u(p), -u^{n-1}(p)))
//   at a source point: u^{n+1} = fma(kappa, amp, u^{n+1})
// where x+/x- = u(p +- m e_x) etc., taken as 0 outside the grid.
//
// Included by kernels_radius.hip, compiled once per radius.
#pragma once

#include "internal.h"

namespace p1310 {

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

// A voffset beyond every buffer window (windows are < 2 GiB): buffer loads
// there return 0 and buffer stores there are dropped. This gives the zero
// ghost layer and the ragged-tile predicate without branches.
constexpr uint32_t kOOB = 0x80000000u;
// Word 3 of a gfx9 raw buffer resource (32-bit data format, no swizzle).
constexpr int kRsrcWord3 = 0x00020000;
// Cache-policy bit for a non-temporal (streaming) access on gfx950.
constexpr int kNT = 2;

template <int VW>
struct alignas(4 * VW) Vec {
    float a[VW];
};

__device__ __forceinline__ rsrc_t make_rsrc(const float *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <int VW, int AUX>
__device__ __forceinline__ Vec<VW> bload(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (VW == 8) {
        Vec<8> v;
        const Vec<4> lo = __builtin_bit_cast(Vec<4>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
        const Vec<4> hi = __builtin_bit_cast(Vec<4>, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16u, soff, AUX));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v.a[e] = lo.a[e];
            v.a[4 + e] = hi.a[e];
        }
        return v;
    } else if constexpr (VW == 4) {
        return __builtin_bit_cast(Vec<4>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
    } else if constexpr (VW == 2) {
        return __builtin_bit_cast(Vec<2>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    } else {
        return __builtin_bit_cast(Vec<1>, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
    }
}

template <int VW, int AUX>
__device__ __forceinline__ void bstore(const Vec<VW> &v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (VW == 8) {
        Vec<4> lo, hi;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            lo.a[e] = v.a[e];
            hi.a[e] = v.a[4 + e];
        }
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, lo), r, voff, soff, AUX);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, hi), r, voff + 16u, soff, AUX);
    } else if constexpr (VW == 4) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, v), r, voff, soff, AUX);
    } else if constexpr (VW == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), r, voff, soff, AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, AUX);
    }
}

template <int VW>
__device__ __forceinline__ Vec<VW> vzero()
{
    Vec<VW> v;
#pragma unroll
    for (int e = 0; e < VW; ++e) v.a[e] = 0.0f;
    return v;
}

// Wavefield storage: FP32, or 16-bit (FP16 / BF16) widened to FP32 on load
// and rounded to nearest even once on store. kappa is always FP32.
template <typename ST>
struct StorageBytes {
    static constexpr int value = sizeof(ST);
};

template <typename ST, int VW, int AUX>
__device__ __forceinline__ Vec<VW> uload(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(ST) == 4) {
        return bload<VW, AUX>(r, voff, soff);
    } else if constexpr (VW == 8) {
        typedef ST s8 __attribute__((ext_vector_type(8)));
        typedef float f8 __attribute__((ext_vector_type(8)));
        const s8 h = __builtin_bit_cast(s8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
        return __builtin_bit_cast(Vec<8>, __builtin_convertvector(h, f8));
    } else if constexpr (VW == 4) {
        typedef ST s4 __attribute__((ext_vector_type(4)));
        typedef float f4 __attribute__((ext_vector_type(4)));
        const s4 h = __builtin_bit_cast(s4, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
        return __builtin_bit_cast(Vec<4>, __builtin_convertvector(h, f4));
    } else if constexpr (VW == 2) {
        typedef ST s2 __attribute__((ext_vector_type(2)));
        typedef float f2 __attribute__((ext_vector_type(2)));
        const s2 h = __builtin_bit_cast(s2, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
        return __builtin_bit_cast(Vec<2>, __builtin_convertvector(h, f2));
    } else {
        Vec<1> v;
        v.a[0] = (float)__builtin_bit_cast(ST, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, AUX));
        return v;
    }
}

template <typename ST, int VW, int AUX>
__device__ __forceinline__ void ustore(const Vec<VW> &v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(ST) == 4) {
        bstore<VW, AUX>(v, r, voff, soff);
    } else if constexpr (VW == 8) {
        typedef ST s8 __attribute__((ext_vector_type(8)));
        typedef float f8 __attribute__((ext_vector_type(8)));
        const s8 h = __builtin_convertvector(__builtin_bit_cast(f8, v), s8);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, h), r, voff, soff, AUX);
    } else if constexpr (VW == 4) {
        typedef ST s4 __attribute__((ext_vector_type(4)));
        typedef float f4 __attribute__((ext_vector_type(4)));
        const s4 h = __builtin_convertvector(__builtin_bit_cast(f4, v), s4);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, h), r, voff, soff, AUX);
    } else if constexpr (VW == 2) {
        typedef ST s2 __attribute__((ext_vector_type(2)));
        typedef float f2 __attribute__((ext_vector_type(2)));
        const s2 h = __builtin_convertvector(__builtin_bit_cast(f2, v), s2);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, h), r, voff, soff, AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (ST)v.a[0]), r, voff, soff, AUX);
    }
}

// Workgroup barrier that orders LDS traffic only: outstanding global loads
// (the next plane's prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Map a workgroup id to a tile id so that each XCD gets a contiguous range
// of tiles. Workgroups are dispatched to the XCDs round-robin by id, so
// without this consecutive (neighbouring) tiles land on different L2s.
__device__ __forceinline__ int xcd_order(int b, int nblk, int nxcd)
{
    const int q = nblk / nxcd, r = nblk % nxcd;
    const int k = b % nxcd, l = b / nxcd;
    return (k < r) ? k * (q + 1) + l : r * (q + 1) + (k - r) * q + l;
}

// ---------------------------------------------------------------------------
// z-march sweep. A workgroup of BX x BY threads owns a TX x TY column of the
// grid (TX = BX*VW along x, TY = BY*RY along y) and marches planes
// z0..z1-1 (z1 - z0 <= dz). Per plane:
//   * the plane's tile and its x/y halo are staged in LDS (double buffered,
//     one barrier per plane); x and y taps are read from LDS;
//   * each thread keeps its points' values of planes z-R..z+R in a register
//     queue of Q = 2R+2 slots, so z taps come from registers and each plane of
//     u^n is fetched from memory once per column;
//   * the next plane's queue entry and halo are fetched before the current
//     plane is computed (software pipelining across the barrier).
// The plane loop is unrolled by Q so that every queue slot index is a
// compile-time constant (no register moves for the shift).
// ---------------------------------------------------------------------------
template <int R, int BX, int BY, int RY, int VW, int PF, typename ST>
__device__ __forceinline__ void zmarch_body(const SweepArgs &a, int b)
{
    constexpr int ES = StorageBytes<ST>::value;  // bytes per wavefield value
    constexpr int NT = BX * BY;
    constexpr int TX = BX * VW, TY = BY * RY;
    constexpr int HX = (VW == 1) ? R : ((R + VW - 1) / VW) * VW;  // x halo, whole vectors
    constexpr int HV = HX / VW;
    constexpr int LW = TX + 2 * HX;        // LDS row length (floats)
    constexpr int LROWS = TY + 2 * R;
    constexpr int LBUF = LROWS * LW + VW;  // + one spare vector for idle halo lanes
    constexpr int Q = 2 * R + 2;
    constexpr int NXH = 2 * TY * HV;       // x-halo vectors per plane
    constexpr int NH = NXH + 2 * R * BX;   // + y-halo vectors
    constexpr int NHI = (NH + NT - 1) / NT;
    static_assert(LBUF % VW == 0, "LDS buffers must stay vector aligned");
    using V = Vec<VW>;

    __shared__ __attribute__((aligned(32))) float lds[2 * LBUF];

    // ---- tile of this workgroup (b = tile id within the grid) --------------
    const int tile_x = b % a.gx;
    const int t2 = b / a.gx;
    const int tile_y = t2 % a.gy;
    const int zc = t2 / a.gy;
    const int x0 = tile_x * TX, y0 = tile_y * TY;
    const int z0 = zc * a.dz;
    const int z1 = min(z0 + a.dz, a.nz);
    const int zlo = max(z0 - R, 0);
    const int zhi = min(z1 + R, a.nz);
    const int64_t plane = (int64_t)a.pitch * a.ny;
    const uint32_t pbytes = (uint32_t)(plane * ES);  // one plane of a wavefield
    const uint32_t kbytes = (uint32_t)(plane * 4);   // one plane of kappa
    const uint32_t win = (uint32_t)(zhi - zlo) * pbytes;
    const uint32_t kwin = (uint32_t)(zhi - zlo) * kbytes;
    const rsrc_t rc = make_rsrc((const float *)((const char *)a.ucur + zlo * plane * ES), win);
    const rsrc_t rp = make_rsrc((const float *)((const char *)a.uprev + zlo * plane * ES), win);
    const rsrc_t rn = make_rsrc((const float *)((char *)a.unext + zlo * plane * ES), win);
    const rsrc_t rk = make_rsrc(a.kappa + zlo * plane, kwin);

    // ---- this thread's points and halo items (same offsets every plane) ----
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int xs = x0 + tx * VW;
    const int yb = y0 + ty * RY;
    uint32_t coff[RY];  // wavefield byte offsets of this thread's rows
    uint32_t koff[RY];  // kappa byte offsets (the same as coff for FP32 storage)
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int y = yb + j;
        const bool in = xs < a.nx && y < a.ny;
        coff[j] = in ? (uint32_t)(y * a.pitch + xs) * (uint32_t)ES : kOOB;
        koff[j] = in ? (uint32_t)(y * a.pitch + xs) * 4u : kOOB;
    }
    uint32_t hg[NHI];
    int hl[NHI];
#pragma unroll
    for (int i = 0; i < NHI; ++i) {
        const int item = tid + i * NT;
        int lrow = 0, lcol = 0, gxx = -1, gyy = -1;
        bool valid = true;
        if (item < NXH) {
            const int r = item / (2 * HV), k = item % (2 * HV);
            const int side = k / HV, v = k % HV;
            lrow = R + r;
            lcol = side ? HX + TX + v * VW : v * VW;
            gyy = y0 + r;
            gxx = side ? x0 + TX + v * VW : x0 - HX + v * VW;
        } else if (item < NH) {
            const int k = item - NXH;
            const int r = k / BX, c = k % BX;
            lrow = (r < R) ? r : TY + r;
            lcol = HX + c * VW;
            gyy = y0 - R + lrow;
            gxx = x0 + c * VW;
        } else {
            valid = false;
        }
        hl[i] = valid ? lrow * LW + lcol : LROWS * LW;
        hg[i] = (valid && gxx >= 0 && gxx < a.nx && gyy >= 0 && gyy < a.ny)
                    ? (uint32_t)(gyy * a.pitch + gxx) * (uint32_t)ES : kOOB;
    }

    // ---- fused single source ------------------------------------------------
    int s_z = -1, s_j = -1, s_e = -1;
    float s_amp = 0.0f;
    if (a.nsrc == 1) {
        const int64_t s = a.src_idx[0];
        if (s >= 0 && s < plane * a.nz) {
            const int sz = (int)(s / plane);
            const int rem = (int)(s - (int64_t)sz * plane);
            const int sy = rem / a.pitch, sx = rem - (rem / a.pitch) * a.pitch;
            if (sz >= z0 && sz < z1 && sx < a.nx) {
                s_z = sz;
                s_amp = a.src_amp[a.it] * a.scale;
                const int dj = sy - yb, de = sx - xs;
                if (dj >= 0 && dj < RY && de >= 0 && de < VW) {
                    s_j = dj;
                    s_e = de;
                }
            }
        }
    }

    V q[Q][RY];
    V hh[2][NHI];
    V pu[2][RY], pk[2][RY];

    auto load_center = [&](V (&dst)[RY], int p) {
        if (p >= 0 && p < a.nz) {
            const uint32_t so = (uint32_t)(p - zlo) * pbytes;
#pragma unroll
            for (int j = 0; j < RY; ++j) dst[j] = uload<ST, VW, 0>(rc, coff[j], so);
        } else {
#pragma unroll
            for (int j = 0; j < RY; ++j) dst[j] = vzero<VW>();
        }
    };
    auto load_halo = [&](V (&dst)[NHI], int p) {
        const uint32_t so = (uint32_t)(p - zlo) * pbytes;
#pragma unroll
        for (int i = 0; i < NHI; ++i) dst[i] = uload<ST, VW, 0>(rc, hg[i], so);
    };
    auto load_uk = [&](V (&du)[RY], V (&dk)[RY], int p) {
        const uint32_t so = (uint32_t)(p - zlo) * pbytes;
        const uint32_t sk = (uint32_t)(p - zlo) * kbytes;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            du[j] = uload<ST, VW, kNT>(rp, coff[j], so);
            dk[j] = bload<VW, kNT>(rk, koff[j], sk);
        }
    };

    // ---- prologue: planes z0-R .. z0+R, halo (and u^{n-1}, kappa) of z0 ----
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) load_center(q[k], z0 - R + k);
    if (z0 < z1) {
        load_halo(hh[0], z0);
        if (PF) load_uk(pu[0], pk[0], z0);
    }

    // Plane z = zb + j keeps plane z+i in queue slot (j + R + i) mod Q.
    for (int zb = z0; zb < z1; zb += Q) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const int z = zb + j;
            if (z >= z1) break;
            const int sc = (j + R) % Q;
            float *buf = lds + (j & 1) * LBUF;
            const uint32_t so = (uint32_t)(z - zlo) * pbytes;
            const uint32_t sk = (uint32_t)(z - zlo) * kbytes;

            // u^{n-1} and kappa of plane z (issued before the prefetch so
            // that waiting for them does not wait for the prefetch).
            V up[RY], kp[RY];
            if (PF) {
#pragma unroll
                for (int jj = 0; jj < RY; ++jj) {
                    up[jj] = pu[j & 1][jj];
                    kp[jj] = pk[j & 1][jj];
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < RY; ++jj) {
                    up[jj] = uload<ST, VW, kNT>(rp, coff[jj], so);
                    kp[jj] = bload<VW, kNT>(rk, koff[jj], sk);
                }
            }

            // Stage plane z: own points and halo.
#pragma unroll
            for (int jj = 0; jj < RY; ++jj)
                *reinterpret_cast<V *>(buf + (R + ty * RY + jj) * LW + HX + tx * VW) = q[sc][jj];
#pragma unroll
            for (int i = 0; i < NHI; ++i) *reinterpret_cast<V *>(buf + hl[i]) = hh[j & 1][i];
            lds_barrier();

            // Prefetch plane z+1: queue entry z+1+R, halo, (u^{n-1}, kappa).
            if (z + 1 < z1) {
                load_center(q[(j + 2 * R + 1) % Q], z + 1 + R);
                load_halo(hh[(j + 1) & 1], z + 1);
                if (PF) load_uk(pu[(j + 1) & 1], pk[(j + 1) & 1], z + 1);
            }

            // y neighbours outside this thread's rows: R rows above, R below.
            V yv[2 * R];
#pragma unroll
            for (int d = 0; d < R; ++d) {
                yv[d] = *reinterpret_cast<const V *>(buf + (ty * RY + d) * LW + HX + tx * VW);
                yv[R + d] = *reinterpret_cast<const V *>(buf + (R + ty * RY + RY + d) * LW + HX + tx * VW);
            }

            V out[RY];
#pragma unroll
            for (int jj = 0; jj < RY; ++jj) {
                const float *row = buf + (R + ty * RY + jj) * LW + tx * VW;
                V xl[HV], xr[HV];
#pragma unroll
                for (int v = 0; v < HV; ++v) {
                    xl[v] = *reinterpret_cast<const V *>(row + v * VW);
                    xr[v] = *reinterpret_cast<const V *>(row + HX + VW + v * VW);
                }
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    const float u0 = q[sc][jj].a[e];
                    float acc = a.c[0] * u0;
#pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        // x window: index w = HX + e +- m into [xl | own | xr].
                        const int wp = HX + e + m, wm = HX + e - m;
                        const float xp = (wp < HX + VW) ? q[sc][jj].a[wp - HX]
                                                        : xr[(wp - HX - VW) / VW].a[(wp - HX - VW) % VW];
                        const float xm = (wm >= HX) ? q[sc][jj].a[wm - HX] : xl[wm / VW].a[wm % VW];
                        const float yp = (jj + m < RY) ? q[sc][jj + m].a[e] : yv[R + jj + m - RY].a[e];
                        const float ym = (jj - m >= 0) ? q[sc][jj - m].a[e] : yv[R + jj - m].a[e];
                        const float zp = q[(j + R + m) % Q][jj].a[e];
                        const float zm = q[(j + R - m + Q) % Q][jj].a[e];
                        const float s = ((xp + xm) + (yp + ym)) + (zp + zm);
                        acc = __builtin_fmaf(a.c[m], s, acc);
                    }
                    out[jj].a[e] = __builtin_fmaf(kp[jj].a[e], acc, __builtin_fmaf(2.0f, u0, -up[jj].a[e]));
                }
            }
            // Source injection: a uniform branch taken on one plane only.
            if (z == s_z) {
#pragma unroll
                for (int jj = 0; jj < RY; ++jj)
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (jj == s_j && e == s_e)
                            out[jj].a[e] = __builtin_fmaf(kp[jj].a[e], s_amp, out[jj].a[e]);
            }
#pragma unroll
            for (int jj = 0; jj < RY; ++jj) ustore<ST, VW, kNT>(out[jj], rn, coff[jj], so);
        }
    }
}

template <int R, int BX, int BY, int RY, int VW, int PF, typename ST>
__global__ void __launch_bounds__(BX * BY) zmarch_kernel(SweepArgs a)
{
    int b = blockIdx.x;
    if (a.xcd > 1) b = xcd_order(b, gridDim.x, a.xcd);
    zmarch_body<R, BX, BY, RY, VW, PF, ST>(a, b);
}

// ---------------------------------------------------------------------------
// Plain tiling: one thread per point, a bx x by x bz workgroup per block of
// the grid, every tap read from memory (caches only). Same arithmetic order.
// ---------------------------------------------------------------------------
template <int R, typename ST>
__global__ void __launch_bounds__(1024) plain_kernel(SweepArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= a.nx || y >= a.ny || z >= a.nz) return;
    const int64_t sy = a.pitch;
    const int64_t sz = (int64_t)a.pitch * a.ny;
    const int64_t p = (int64_t)z * sz + (int64_t)y * sy + x;
    const ST *u = (const ST *)a.ucur;
    const float u0 = (float)u[p];
    float acc = a.c[0] * u0;
#pragma unroll
    for (int m = 1; m <= R; ++m) {
        const float xp = (x + m < a.nx) ? (float)u[p + m] : 0.0f;
        const float xm = (x - m >= 0) ? (float)u[p - m] : 0.0f;
        const float yp = (y + m < a.ny) ? (float)u[p + m * sy] : 0.0f;
        const float ym = (y - m >= 0) ? (float)u[p - m * sy] : 0.0f;
        const float zp = (z + m < a.nz) ? (float)u[p + m * sz] : 0.0f;
        const float zm = (z - m >= 0) ? (float)u[p - m * sz] : 0.0f;
        const float s = ((xp + xm) + (yp + ym)) + (zp + zm);
        acc = __builtin_fmaf(a.c[m], s, acc);
    }
    const float k = a.kappa[p];
    float o = __builtin_fmaf(k, acc, __builtin_fmaf(2.0f, u0, -(float)((const ST *)a.uprev)[p]));
    if (a.nsrc == 1 && a.src_idx[0] == p) o = __builtin_fmaf(k, a.src_amp[a.it] * a.scale, o);
    ((ST *)a.unext)[p] = (ST)o;
}

}  // namespace p1310
