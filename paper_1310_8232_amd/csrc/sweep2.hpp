// Two-step (temporally blocked) z-march kernel; shares the helpers of the
// one-step sweep (sweep.hpp).
#pragma once

#include "sweep.hpp"

namespace p1310 {

// ---------------------------------------------------------------------------
// Two-step z-march (blocking in time as well as in space). One launch reads
// u^n, u^{n-1}, kappa and writes u^{n+1} and u^{n+2} to two further buffers
// (the inputs stay untouched: neighbouring workgroups read them in their
// halos). A workgroup of BX x BY threads covers an extended tile E of
// (BX*VW) x BY points; its own tile is E without an R-wide ring
// ((BX*VW - 2HX) x (BY - 2R)). Iteration z of the march:
//   step 1: u^{n+1} at plane z on all of E, exactly as the one-step march
//           (u^n staged in LDS with its halo, register queue q1 of u^n);
//           E's ring duplicates the neighbours' work so that step 2 needs no
//           exchange; own points are stored;
//   step 2: u^{n+2} at plane z' = z - R - 1 on the own tile: x/y taps of
//           u^{n+1}(z') from a second LDS plane staged in the same iteration,
//           z taps from a register queue q2 of u^{n+1}, u^n(z') from q1.
// Both LDS planes are double buffered and staged before the iteration's one
// barrier. A chunk [z0, z1) of output planes runs step 1 over planes
// z0-R .. z1+R-1 and one more iteration for the last step-2 plane. PF = 1
// loads u^{n-1} and kappa one plane ahead. kappa for step 2 is not loaded
// again: each lane keeps the kappa its step 1 loaded for the last R + 1
// planes in a register queue, and step 2's plane z' = z - R - 1 is the oldest
// of them. u^{n-1} and kappa are read over all of E, so the ring positions
// are read by neighbouring workgroups too: those loads use the default
// (cached) policy. The stencil sums run one radius at a time (the y pair of
// radius m read from LDS and consumed before radius m + 1), which keeps the
// register peak low; the per-point operation order is the canonical one, so
// the results are the bits of two one-step sweeps. Algorithmic HBM traffic:
// 20 B per point for two updates. Edge pacing (SweepArgs::pace): with the XCD
// order, the tiles of one XCD share the halo lines of their neighbours in its
// L2 only while they march near the same plane; the first and last tile
// columns read fewer bytes and would run ahead, so they pause for a fixed
// time per plane (a timing option only: the arithmetic is untouched).
// ---------------------------------------------------------------------------
template <int R, int BX, int BY, int VW, int PF, typename ST>
__device__ __forceinline__ void zmarch2_body(const SweepArgs &a, int b)
{
    constexpr int ES = StorageBytes<ST>::value;
    constexpr int NT = BX * BY;
    constexpr int EX = BX * VW, EY = BY;
    constexpr int HX = (VW == 1) ? R : ((R + VW - 1) / VW) * VW;
    constexpr int HV = HX / VW;
    constexpr int OX = EX - 2 * HX, OY = EY - 2 * R;
    static_assert(OX > 0 && OY > 0, "extended tile too small for the radius");
    // LDS row of the u^n plane: EX + 2HX floats, padded when a row of BX
    // threads is not a whole number of 16-lane groups (BX = 18, 8): then a
    // 16-lane b128 access spans two rows, and (LW/4 - BX) % 16 == 0 makes the
    // second row continue the first one's 16-byte bank-group sequence, so
    // the access is conflict-free.
    constexpr int LW0 = EX + 2 * HX;
    constexpr bool kStraddle = VW == 4 && (BX % 16) != 0;
    constexpr int LW = kStraddle ? LW0 + ((((BX - LW0 / 4) % 16) + 16) % 16) * 4 : LW0;
    static_assert(!kStraddle || ((LW / 4 - BX) % 16 == 0 && LW % 4 == 0), "LDS row padding");
    constexpr int LROWS = EY + 2 * R;
    constexpr int LBUF = LROWS * LW + VW;
    constexpr int L2BUF = EY * EX;
    constexpr int Q = 2 * R + 2;
    constexpr int NXH = 2 * EY * HV;
    constexpr int NH = NXH + 2 * R * BX;
    constexpr int NHI = (NH + NT - 1) / NT;
    static_assert(LBUF % VW == 0, "LDS buffers must stay vector aligned");
    static_assert(L2BUF % VW == 0, "LDS buffers must stay vector aligned");
    using V = Vec<VW>;

    __shared__ __attribute__((aligned(16))) float lds1[2 * LBUF];
    __shared__ __attribute__((aligned(16))) float lds2[2 * L2BUF];

    const int tile_x = b % a.gx;
    const int t2 = b / a.gx;
    const int tile_y = t2 % a.gy;
    const int zc = t2 / a.gy;
    const int x0 = tile_x * OX, y0 = tile_y * OY;  // own tile origin
    const int ex0 = x0 - HX, ey0 = y0 - R;         // extended tile origin
    const int z0 = zc * a.dz;
    const int z1 = min(z0 + a.dz, a.nz);
    const int zs = z0 - R, ze = z1 + R;            // step-1 planes [zs, ze)
    // Edge pacing: the first and last tile columns read fewer bytes (their
    // out-of-grid halo costs none) and would march ahead of their neighbours.
    const int pace = (a.gx >= 3 && (tile_x == 0 || tile_x == a.gx - 1)) ? a.pace : 0;
    const int zlo = max(z0 - 2 * R, 0);
    const int zhi = min(z1 + 2 * R, a.nz);
    const int64_t plane = (int64_t)a.pitch * a.ny;
    const uint32_t pbytes = (uint32_t)(plane * ES);
    const uint32_t kbytes = (uint32_t)(plane * 4);
    const uint32_t win = (uint32_t)(zhi - zlo) * pbytes;
    const uint32_t kwin = (uint32_t)(zhi - zlo) * kbytes;
    const rsrc_t rc = make_rsrc((const float *)((const char *)a.ucur + zlo * plane * ES), win);
    const rsrc_t rp = make_rsrc((const float *)((const char *)a.uprev + zlo * plane * ES), win);
    const rsrc_t rn1 = make_rsrc((const float *)((char *)a.unext + zlo * plane * ES), win);
    const rsrc_t rn2 = make_rsrc((const float *)((char *)a.unext2 + zlo * plane * ES), win);
    const rsrc_t rk = make_rsrc(a.kappa + zlo * plane, kwin);

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int xs = ex0 + tx * VW;
    const int yy = ey0 + ty;
    const bool in = xs >= 0 && xs < a.nx && yy >= 0 && yy < a.ny;
    const bool own = tx >= HV && tx < BX - HV && ty >= R && ty < BY - R;
    const uint32_t coff = in ? (uint32_t)(yy * a.pitch + xs) * (uint32_t)ES : kOOB;
    const uint32_t koff = in ? (uint32_t)(yy * a.pitch + xs) * 4u : kOOB;
    const uint32_t soff = own ? coff : kOOB;  // stores: own points only

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
            lcol = side ? HX + EX + v * VW : v * VW;
            gyy = ey0 + r;
            gxx = side ? ex0 + EX + v * VW : ex0 - HX + v * VW;
        } else if (item < NH) {
            const int k = item - NXH;
            const int r = k / BX, c = k % BX;
            lrow = (r < R) ? r : EY + r;
            lcol = HX + c * VW;
            gyy = ey0 - R + lrow;
            gxx = ex0 + c * VW;
        } else {
            valid = false;
        }
        hl[i] = valid ? lrow * LW + lcol : LROWS * LW;
        hg[i] = (valid && gxx >= 0 && gxx < a.nx && gyy >= 0 && gyy < a.ny)
                    ? (uint32_t)(gyy * a.pitch + gxx) * (uint32_t)ES : kOOB;
    }

    // Single source at steps it (into u^{n+1}) and it+1 (into u^{n+2}).
    int s_z = -1, s_e = -1;
    float s_amp1 = 0.0f, s_amp2 = 0.0f;
    if (a.nsrc == 1) {
        const int64_t s = a.src_idx[0];
        if (s >= 0 && s < plane * a.nz) {
            const int sz = (int)(s / plane);
            const int rem = (int)(s - (int64_t)sz * plane);
            const int sy = rem / a.pitch, sx = rem - (rem / a.pitch) * a.pitch;
            if (sz >= zs && sz < ze && sx < a.nx) {
                s_z = sz;
                s_amp1 = a.src_amp[a.it] * a.scale;
                s_amp2 = a.src_amp[a.it + 1] * a.scale;
                const int de = sx - xs;
                if (sy == yy && de >= 0 && de < VW) s_e = de;
            }
        }
    }

    V q1[Q], q2[Q];
    V hh[2][NHI];
    V upf[2], kpf[2];  // PF: u^{n-1} and kappa of planes z (slot z & 1) and z + 1
    constexpr int KQ = R + 1;
    V kq2[KQ];         // kappa of the last R + 1 step-1 planes: plane p in slot (p - zs) mod (R + 1)

    auto plane_ok = [&](int p) { return p >= 0 && p < a.nz; };
    // A plane outside the grid is read through an out-of-range vector offset
    // (and a zero scalar offset), which returns zeros: the loads need no
    // branch and no zeroing moves.
    auto load_center = [&](V &dst, int p) {
        const bool ok = plane_ok(p);
        dst = uload<ST, VW, 0>(rc, ok ? coff : kOOB, ok ? (uint32_t)(p - zlo) * pbytes : 0u);
    };
    auto load_halo = [&](V (&dst)[NHI], int p) {
        const bool ok = plane_ok(p);
        const uint32_t so = ok ? (uint32_t)(p - zlo) * pbytes : 0u;
#pragma unroll
        for (int i = 0; i < NHI; ++i) dst[i] = uload<ST, VW, 0>(rc, ok ? hg[i] : kOOB, so);
    };
    auto load_pk = [&](V &u, V &k, int p) {
        const bool ok = plane_ok(p);
        u = uload<ST, VW, 0>(rp, ok ? coff : kOOB, ok ? (uint32_t)(p - zlo) * pbytes : 0u);
        k = bload<VW, 0>(rk, ok ? koff : kOOB, ok ? (uint32_t)(p - zlo) * kbytes : 0u);
    };

    // Prologue: u^n planes zs-R .. zs+R (queue slots 0..2R), halo of plane zs.
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) load_center(q1[k], zs - R + k);
#pragma unroll
    for (int k = 0; k < Q; ++k) q2[k] = vzero<VW>();
    load_halo(hh[0], zs);
    if (PF) load_pk(upf[0], kpf[0], zs);
#pragma unroll
    for (int k = 0; k < KQ; ++k) kq2[k] = vzero<VW>();

    // Iteration z = zb + j keeps plane p of u^n and of u^{n+1} in queue slot
    // (p - zs + R) mod Q: plane z in slot (j + R) mod Q, plane z' = z - R - 1
    // in slot (j - 1) mod Q, which is also where plane z + R + 1 of u^n goes.
    for (int zb = zs; zb <= ze; zb += Q) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const int z = zb + j;
            if (z > ze) break;
            const int sc = (j + R) % Q;
            const int sq = (j + Q - 1) % Q;
            const int zq = z - R - 1;
            const bool st1 = z < ze;
            const bool st2 = zq >= z0 && zq < z1;
            float *buf1 = lds1 + (j & 1) * LBUF;
            float *buf2 = lds2 + (j & 1) * L2BUF;
            if (pace) {  // uniform for the workgroup; a pause of about 4 * pace * 64 cycles
                switch (pace) {
                case 1: __builtin_amdgcn_s_sleep(4); break;
                case 2: __builtin_amdgcn_s_sleep(8); break;
                case 3: __builtin_amdgcn_s_sleep(12); break;
                case 4: __builtin_amdgcn_s_sleep(16); break;
                case 5: __builtin_amdgcn_s_sleep(20); break;
                case 6: __builtin_amdgcn_s_sleep(24); break;
                default: __builtin_amdgcn_s_sleep(28); break;
                }
            }

            // u^{n-1} and kappa of plane z on E.
            V up, kp;
            if (PF) {
                up = upf[j & 1];
                kp = kpf[j & 1];
            } else if (st1) {
                load_pk(up, kp, z);
            }

            // Stage u^n plane z with its halo and u^{n+1} plane z'.
            if (st1) {
                *reinterpret_cast<V *>(buf1 + (R + ty) * LW + HX + tx * VW) = q1[sc];
#pragma unroll
                for (int i = 0; i < NHI; ++i) *reinterpret_cast<V *>(buf1 + hl[i]) = hh[j & 1][i];
            }
            if (st2) *reinterpret_cast<V *>(buf2 + ty * EX + tx * VW) = q2[sq];
            lds_barrier();

            const V un = q1[sq];  // u^n(z'), before the slot is refilled
            if (z + 1 < ze) {
                load_center(q1[sq], z + 1 + R);
                load_halo(hh[(j + 1) & 1], z + 1);
                if (PF) load_pk(upf[(j + 1) & 1], kpf[(j + 1) & 1], z + 1);
            }

            // Step 2: u^{n+2}(z') on the own tile. Every lane runs it in every
            // iteration (no divergent branch, so the compiler schedules it
            // together with step 1): ring lanes read the LDS taps of the
            // nearest own position and planes outside the chunk compute on
            // stale LDS data; neither is stored (the store offset is out of
            // the window for them).
            {
                const int tyc = min(max(ty, R), BY - R - 1), txc = min(max(tx, HV), BX - HV - 1);
                const float *row = buf2 + tyc * EX + txc * VW - HX;
                V xl[HV], xr[HV];
#pragma unroll
                for (int v = 0; v < HV; ++v) {
                    xl[v] = *reinterpret_cast<const V *>(row + v * VW);
                    xr[v] = *reinterpret_cast<const V *>(row + HX + VW + v * VW);
                }
                const V &c1 = q2[sq];  // u^{n+1}(z')
                const V kq = kq2[j % KQ];  // kappa(z'), loaded by step 1 R + 1 iterations ago
                float acc[VW];
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] = a.c[0] * c1.a[e];
                // One radius at a time: its y pair is read from LDS and used
                // before the next radius's, so the taps of one radius are live
                // at a time (the per-point operation order is unchanged).
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    const V yp = *reinterpret_cast<const V *>(buf2 + (tyc + m) * EX + txc * VW);
                    const V ym = *reinterpret_cast<const V *>(buf2 + (tyc - m) * EX + txc * VW);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        const int wp = HX + e + m, wm = HX + e - m;
                        const float xp = (wp < HX + VW) ? c1.a[wp - HX]
                                                        : xr[(wp - HX - VW) / VW].a[(wp - HX - VW) % VW];
                        const float xm = (wm >= HX) ? c1.a[wm - HX] : xl[wm / VW].a[wm % VW];
                        const float zp = q2[(j + Q - 1 + m) % Q].a[e];
                        const float zm = q2[(j + Q - 1 - m) % Q].a[e];
                        const float s = ((xp + xm) + (yp.a[e] + ym.a[e])) + (zp + zm);
                        acc[e] = __builtin_fmaf(a.c[m], s, acc[e]);
                    }
                }
                V out;
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    out.a[e] = __builtin_fmaf(kq.a[e], acc[e], __builtin_fmaf(2.0f, c1.a[e], -un.a[e]));
                if (zq == s_z) {
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (e == s_e) out.a[e] = __builtin_fmaf(kq.a[e], s_amp2, out.a[e]);
                }
                ustore<ST, VW, kNT>(out, rn2, st2 ? soff : kOOB, st2 ? (uint32_t)(zq - zlo) * pbytes : 0u);
            }

            // Step 1: u^{n+1}(z) on E.
            if (st1) {
                const float *row = buf1 + (R + ty) * LW + tx * VW;
                V xl[HV], xr[HV];
#pragma unroll
                for (int v = 0; v < HV; ++v) {
                    xl[v] = *reinterpret_cast<const V *>(row + v * VW);
                    xr[v] = *reinterpret_cast<const V *>(row + HX + VW + v * VW);
                }
                float acc[VW];
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] = a.c[0] * q1[sc].a[e];
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    const V yp = *reinterpret_cast<const V *>(buf1 + (R + ty + m) * LW + HX + tx * VW);
                    const V ym = *reinterpret_cast<const V *>(buf1 + (R + ty - m) * LW + HX + tx * VW);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        const int wp = HX + e + m, wm = HX + e - m;
                        const float xp = (wp < HX + VW) ? q1[sc].a[wp - HX]
                                                        : xr[(wp - HX - VW) / VW].a[(wp - HX - VW) % VW];
                        const float xm = (wm >= HX) ? q1[sc].a[wm - HX] : xl[wm / VW].a[wm % VW];
                        const float zp = q1[(j + R + m) % Q].a[e];
                        const float zm = q1[(j + R - m + Q) % Q].a[e];
                        const float s = ((xp + xm) + (yp.a[e] + ym.a[e])) + (zp + zm);
                        acc[e] = __builtin_fmaf(a.c[m], s, acc[e]);
                    }
                }
                V out;
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    out.a[e] = __builtin_fmaf(kp.a[e], acc[e], __builtin_fmaf(2.0f, q1[sc].a[e], -up.a[e]));
                if (z == s_z) {
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (e == s_e) out.a[e] = __builtin_fmaf(kp.a[e], s_amp1, out.a[e]);
                }
                q2[sc] = out;
                kq2[j % KQ] = kp;
                if (z >= z0 && z < z1) ustore<ST, VW, kNT>(out, rn1, soff, (uint32_t)(z - zlo) * pbytes);
            }
        }
    }
}

template <int R, int BX, int BY, int VW, int PF, typename ST>
__global__ void __launch_bounds__(BX * BY) zmarch2_kernel(SweepArgs a)
{
    int b = blockIdx.x;
    if (a.xcd > 1) b = xcd_order(b, gridDim.x, a.xcd);
    zmarch2_body<R, BX, BY, VW, PF, ST>(a, b);
}

}  // namespace p1310
