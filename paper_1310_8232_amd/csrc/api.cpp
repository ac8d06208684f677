// C-ABI runtime: context, validation, dispatch, the blocksize search and its
// cache. Declarations and contracts: include/stencil.h.
#include "../../include/stencil.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <initializer_list>
#include <vector>

#include "internal.h"

using p1310::SweepArgs;
using p1310::Z2Variant;
using p1310::ZVariant;

struct stencil_ctx {
    stencil_desc d;
    int64_t pitch = 0;     // row stride in values (d.pitch, or nx when that is 0)
    int R = 4;
    int st = p1310::kF32;  // wavefield storage
    int es = 4;            // bytes per wavefield value
    float scale = 1.0f;    // storage scale (power of two)
    float cf[p1310::kMaxRadius + 1] = {};  // 3*c_0, c_1..c_R in FP32
    stencil_tile tile = {};   // one-step sweeps
    stencil_tile tile2 = {};  // two-step sweeps (kind STENCIL_TILE_ZMARCH2)
    std::string err;
};

struct stencil_batch {
    struct Shot {
        stencil_ctx *ctx;
        const float *kappa;
        void *u_a, *u_b;
        stencil_src src;
        stencil_tile tile;
    };
    struct Group {
        const p1310::ZVariant *v;
        int xcd;
        int nshots;
        int blocks;
        p1310::SweepArgs *tab[2];  // device: step parity 0 / 1
        int *begin;                // device: first workgroup of each shot
    };
    std::vector<Shot> shots;
    std::vector<Group> groups;
    std::vector<int> solo;  // shots launched on their own (plain tiles)
    int64_t it0 = 0;
    int64_t nt_min = 0;     // smallest source length (steps must stay below it)
    void *dmem = nullptr;
    int device = 0;
    bool in_static = false;    // table in the device's static table (no hipMalloc)
    uint64_t generation = 0;   // static table contents this batch was built with
};

namespace {

constexpr int kXcds = 8;  // MI355X: 256 CUs in 8 accelerator complex dies
constexpr int64_t kWindowLimit = (int64_t)1 << 31;

// A 1-D launch: at most 2^31 - 1 workgroups and 2^32 - 1 work-items (the
// dispatch packet's grid size is a 32-bit count of work-items).
bool launch_fits(int64_t blocks, int threads)
{
    return blocks >= 1 && blocks <= 0x7fffffff && blocks * threads <= (int64_t)0xffffffff;
}

// ---------------------------------------------------------------------------
// Exact rational weights of the order-2R central second difference.
// c_m = 2 (-1)^{m+1} (R!)^2 / (m^2 (R-m)! (R+m)!), c_0 = -2 sum c_m.
// ---------------------------------------------------------------------------
struct Rat {
    long long n, d;
};

long long gcdll(long long a, long long b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        long long t = a % b;
        a = b;
        b = t;
    }
    return a ? a : 1;
}

Rat rnorm(Rat r)
{
    if (r.d < 0) {
        r.n = -r.n;
        r.d = -r.d;
    }
    long long g = gcdll(r.n, r.d);
    return {r.n / g, r.d / g};
}

Rat radd(Rat a, Rat b)
{
    long long g = gcdll(a.d, b.d);
    return rnorm({a.n * (b.d / g) + b.n * (a.d / g), a.d / g * b.d});
}

Rat rmul(Rat a, long long k) { return rnorm({a.n * k, a.d}); }

long long factll(int k)
{
    long long f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

bool radius_ok(int R) { return R >= 3 && R <= p1310::kMaxRadius; }

void weights(int R, Rat *c)
{
    const long long rf = factll(R);
    Rat sum = {0, 1};
    for (int m = 1; m <= R; ++m) {
        c[m] = rnorm({(m % 2 ? 2 : -2) * rf * rf, (long long)m * m * factll(R - m) * factll(R + m)});
        sum = radd(sum, c[m]);
    }
    c[0] = rmul(sum, -2);
}

double rat_to_double(Rat r) { return (double)r.n / (double)r.d; }

double cfl_limit_of(int R)
{
    Rat c[p1310::kMaxRadius + 1];
    weights(R, c);
    Rat s = c[0];
    for (int m = 1; m <= R; ++m) s = radd(s, rmul(c[m], (m % 2) ? -2 : 2));
    return 2.0 / std::sqrt(3.0 * std::fabs(rat_to_double(s)));
}

// Last error of calls made without a context (batches, misfit, probe), per thread.
thread_local std::string g_err;

// STENCIL_LOG set to anything but "" or "0": one line per context creation
// and per search on stderr (read at each such call, never in a step).
bool log_on()
{
    const char *e = std::getenv("STENCIL_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
}

const char *storage_name(int st)
{
    static const char *kst[] = {"f32", "f16", "bf16"};
    return (st >= 0 && st <= 2) ? kst[st] : "?";
}

std::string tile_text(const stencil_tile &t)
{
    char b[160];
    static const char *kind[] = {"auto", "plain", "zmarch", "zmarch2"};
    const int n = std::snprintf(b, sizeof b, "%s %dx%d ry%d dz%d vw%d xcd%d pf%d",
                                (t.kind >= 0 && t.kind <= 3) ? kind[t.kind] : "?", t.bx, t.by, t.ry, t.dz, t.vw, t.xcd,
                                t.kind == STENCIL_TILE_ZMARCH2 ? (t.pf & 1) : t.pf);
    if (t.kind == STENCIL_TILE_ZMARCH2 && (t.pf >> 1) && n > 0 && n < (int)sizeof b)
        std::snprintf(b + n, sizeof b - n, " pace%d", t.pf >> 1);
    return b;
}

stencil_status fail(stencil_ctx *ctx, stencil_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_err = msg;
    return st;
}

size_t round256(size_t n) { return (n + 255) / 256 * 256; }

// Values of one field as stored: pitch * ny * nz (the padding included).
int64_t nstore(const stencil_ctx *c) { return c->pitch * c->d.ny * c->d.nz; }

// A vector of vw values must neither straddle the end of a row's grid points
// nor leave the row's alignment: vw divides nx and the pitch.
bool vw_fits(const stencil_ctx *c, int vw) { return c->d.nx % vw == 0 && c->pitch % vw == 0; }

bool vec4_ok(const stencil_ctx *c) { return vw_fits(c, 4); }

bool has_vw(const stencil_ctx *ctx, int vw)
{
    for (int i = 0; i < p1310::zmarch_variant_count(); ++i) {
        const ZVariant *v = p1310::zmarch_variant(i);
        if (v->R == ctx->R && v->st == ctx->st && v->vw == vw) return true;
    }
    return false;
}

// Widest x vector that divides nx and has compiled one-step kernels.
int auto_vw(const stencil_ctx *ctx)
{
    if (vw_fits(ctx, 8) && has_vw(ctx, 8)) return 8;
    if (vw_fits(ctx, 4)) return 4;
    if (vw_fits(ctx, 2) && has_vw(ctx, 2)) return 2;
    return 1;
}

// Vector accesses of vw values need kappa on 4*vw-byte boundaries and the
// wavefields on vw-value boundaries.
bool vec_aligned(const stencil_ctx *ctx, int vw, const void *kappa, std::initializer_list<const void *> fields)
{
    if (vw <= 1) return true;
    if ((uintptr_t)kappa & (uintptr_t)(4 * vw - 1)) return false;
    for (const void *f : fields)
        if ((uintptr_t)f & (uintptr_t)(vw * ctx->es - 1)) return false;
    return true;
}

const ZVariant *find_variant(const stencil_ctx *ctx, const stencil_tile &t)
{
    for (int i = 0; i < p1310::zmarch_variant_count(); ++i) {
        const ZVariant *v = p1310::zmarch_variant(i);
        if (v->R == ctx->R && v->st == ctx->st && v->bx == t.bx && v->by == t.by && v->ry == t.ry && v->vw == t.vw &&
            v->pf == t.pf)
            return v;
    }
    return nullptr;
}

const Z2Variant *find_variant2(const stencil_ctx *ctx, const stencil_tile &t)
{
    for (int i = 0; i < p1310::zmarch2_variant_count(); ++i) {
        const Z2Variant *v = p1310::zmarch2_variant(i);
        if (v->R == ctx->R && v->st == ctx->st && v->bx == t.bx && v->by == t.by && v->vw == t.vw &&
            v->pf == (t.pf & 1))
            return v;
    }
    return nullptr;
}

// Checks a concrete tile against the grid; on success fills *norm with the
// normalised tile (vw picked, xcd clamped).
stencil_status check_tile(stencil_ctx *ctx, const stencil_tile &in, stencil_tile *norm)
{
    stencil_tile t = in;
    const stencil_desc &d = ctx->d;
    if (t.kind == STENCIL_TILE_PLAIN) {
        if (t.bx < 1 || t.by < 1 || t.dz < 1 || (int64_t)t.bx * t.by * t.dz > 1024)
            return fail(ctx, STENCIL_EUNSUPPORTED, "plain tile needs bx, by, dz >= 1 and bx*by*dz <= 1024");
        if ((d.ny + t.by - 1) / t.by > 65535 || (d.nz + t.dz - 1) / t.dz > 65535 ||
            (d.nx + t.bx - 1) / t.bx > 0x7fffffff)
            return fail(ctx, STENCIL_EUNSUPPORTED, "plain tile: launch grid too large for this grid");
        t.ry = 1;
        t.vw = 1;
        t.xcd = 0;
        t.pf = 0;
        *norm = t;
        return STENCIL_OK;
    }
    if (t.kind == STENCIL_TILE_ZMARCH2) {
        if (t.vw == 0) t.vw = vec4_ok(ctx) ? 4 : 1;
        if (t.vw < 1 || !vw_fits(ctx, t.vw)) return fail(ctx, STENCIL_EUNSUPPORTED, "vw must divide nx and the pitch");
        if (t.pf < 0 || t.pf > 15)
            return fail(ctx, STENCIL_EUNSUPPORTED, "two-step pf: bit 0 prefetch, bits 1-3 edge pacing (0..15)");
        t.ry = 1;
        const Z2Variant *v = find_variant2(ctx, t);
        if (!v) return fail(ctx, STENCIL_EUNSUPPORTED, "no compiled two-step kernel for this (bx, by, vw), radius, storage");
        if (t.dz < 1) return fail(ctx, STENCIL_EUNSUPPORTED, "dz must be >= 1");
        if (t.dz > d.nz) t.dz = (int32_t)d.nz;
        if ((t.dz + 4 * ctx->R) * ctx->pitch * d.ny * 4 >= kWindowLimit)
            return fail(ctx, STENCIL_EUNSUPPORTED, "two-step window (dz + 4R planes) must stay below 2 GiB; lower dz");
        const int64_t gx = (d.nx + v->own_x - 1) / v->own_x, gy = (d.ny + v->own_y - 1) / v->own_y;
        if (!launch_fits(gx * gy * ((d.nz + t.dz - 1) / t.dz), v->threads))
            return fail(ctx, STENCIL_EUNSUPPORTED, "launch too large (over 2^31-1 workgroups or 2^32-1 work-items); raise dz");
        t.xcd = t.xcd ? kXcds : 0;
        *norm = t;
        return STENCIL_OK;
    }
    if (t.kind != STENCIL_TILE_ZMARCH) return fail(ctx, STENCIL_EUNSUPPORTED, "unknown tile kind");
    if (t.vw == 0) t.vw = auto_vw(ctx);
    if (t.vw < 1 || !vw_fits(ctx, t.vw)) return fail(ctx, STENCIL_EUNSUPPORTED, "vw must divide nx and the pitch");
    const ZVariant *zv = find_variant(ctx, t);
    if (!zv) return fail(ctx, STENCIL_EUNSUPPORTED, "no compiled z-march kernel for this (bx, by, ry, vw, pf) and radius");
    if (t.dz < 1) return fail(ctx, STENCIL_EUNSUPPORTED, "dz must be >= 1");
    if (t.dz > d.nz) t.dz = (int32_t)d.nz;
    const int64_t plane_bytes = ctx->pitch * d.ny * 4;
    if ((t.dz + 2 * ctx->R) * plane_bytes >= kWindowLimit)
        return fail(ctx, STENCIL_EUNSUPPORTED, "z-march window (dz + 2R planes) must stay below 2 GiB; lower dz");
    const int64_t gx = (d.nx + (int64_t)t.bx * t.vw - 1) / ((int64_t)t.bx * t.vw);
    const int64_t gy = (d.ny + (int64_t)t.by * t.ry - 1) / ((int64_t)t.by * t.ry);
    const int64_t gz = (d.nz + t.dz - 1) / t.dz;
    if (!launch_fits(gx * gy * gz, zv->threads))
        return fail(ctx, STENCIL_EUNSUPPORTED, "launch too large (over 2^31-1 workgroups or 2^32-1 work-items); raise dz");
    t.xcd = t.xcd ? kXcds : 0;
    *norm = t;
    return STENCIL_OK;
}

bool zmarch_possible(const stencil_ctx *ctx)
{
    return (1 + 2 * ctx->R) * ctx->pitch * ctx->d.ny * 4 < kWindowLimit;
}

// Deepest march whose window of dz + halo_planes planes stays below 2 GiB.
int32_t max_dz(const stencil_ctx *ctx, int halo_planes)
{
    const int64_t plane_bytes = ctx->pitch * ctx->d.ny * 4;
    const int64_t dz = (kWindowLimit - 1) / plane_bytes - halo_planes;
    return dz < 1 ? 0 : (int32_t)std::min<int64_t>(dz, 1 << 30);
}

// The untuned tile. Shapes from full searches at 64^3 .. 1024x1024x512
// (R = 3, 4, 5; FP32): 256 x 16 points (64 x 8 threads, two rows each) for
// widths that are multiples of 256 from 512 up, 128 x 8 points from 128 up,
// 64 x 8 below; the march depth is the deepest of 256, 128, ..., 4 planes
// that still gives at least 512 workgroups (two per CU), so small grids fill
// the device with shallow marches and large ones keep the z halo small.
// Against the searched tile at those shapes: 1.00 at 512^3 (R = 4, 5), 10%
// slower on average, 33% at most (unaligned widths of 200 and 300).
stencil_tile default_tile(const stencil_ctx *ctx)
{
    stencil_tile t = {};
    if (!zmarch_possible(ctx)) {
        t.kind = STENCIL_TILE_PLAIN;
        t.bx = 64;
        t.by = 4;
        t.dz = 1;
        return t;
    }
    t.kind = STENCIL_TILE_ZMARCH;
    const int64_t nx = ctx->d.nx, ny = ctx->d.ny, nz = ctx->d.nz;
    const int vw = auto_vw(ctx);
    if (vw >= 4) {
        t.vw = 4;
        t.by = 8;
        if (nx >= 512 && nx % 256 == 0) {
            t.bx = 64;
            t.ry = 2;
        } else {
            t.bx = nx >= 128 ? 32 : 16;
            t.ry = 1;
        }
    } else if (vw == 2) {
        t.bx = 64;
        t.by = 4;
        t.ry = 1;
        t.vw = 2;
    } else {
        t.bx = 64;
        t.by = 4;
        t.ry = ctx->st == p1310::kF32 ? 2 : 1;
        t.vw = 1;
    }
    const int64_t cols = ((nx + (int64_t)t.bx * t.vw - 1) / ((int64_t)t.bx * t.vw)) *
                         ((ny + (int64_t)t.by * t.ry - 1) / ((int64_t)t.by * t.ry));
    int32_t dz = 4;
    for (int32_t d : {256, 128, 64, 32, 16, 8, 4})
        if (cols * ((nz + d - 1) / d) >= 512) {
            dz = d;
            break;
        }
    t.dz = std::min<int32_t>(dz, max_dz(ctx, 2 * ctx->R));
    t.xcd = 1;
    t.pf = 0;
    return t;
}

stencil_tile default_tile2(const stencil_ctx *ctx)
{
    stencil_tile t = {};
    t.kind = STENCIL_TILE_ZMARCH2;
    if (vec4_ok(ctx)) {
        // 18 x 40 is not compiled for R = 5 (it would spill registers).
        t.bx = ctx->R <= 4 ? 18 : 16;
        t.by = ctx->R <= 4 ? 40 : 32;
        t.vw = 4;
    } else {
        t.bx = 32;
        t.by = 16;
        t.vw = 1;
    }
    t.ry = 1;
    t.dz = std::min<int32_t>(128, max_dz(ctx, 4 * ctx->R));  // 0 (rejected) when no window fits
    t.xcd = 1;
    return t;
}

// --------------------------------------------------------------------------
// Tune cache: one line per entry,
//   v2 <build id> R<r> <storage> <nx> <ny> <nz> <pitch> <kind> <bx> <by> <ry> <dz> <vw> <xcd> <pf> <min_ms>
//   <actual_ms>
// where the build id (stencil_build_id) names the offload architecture, the
// HIP version the kernels were compiled with, the HIP runtime in use and a
// hash of the kernel and runtime sources. An entry measured with other code
// (another build id, or the unversioned format of earlier builds) is
// ignored: its tile may no longer be the fastest. The last matching line wins.
// --------------------------------------------------------------------------
#ifndef P1310_SOURCE_HASH
#define P1310_SOURCE_HASH "unknown"
#endif
#ifndef P1310_ARCH
#define P1310_ARCH "gfx950"
#endif

const std::string &build_id()
{
    static const std::string id = [] {
        int rt = 0;
        if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = -1;
        char b[160];
        std::snprintf(b, sizeof b, "%s/hip%d/rt%d/src%s", P1310_ARCH, (int)HIP_VERSION, rt, P1310_SOURCE_HASH);
        return std::string(b);
    }();
    return id;
}

bool cache_lookup(const char *path, const stencil_ctx *ctx, bool two, stencil_tile *t, double *mn, double *act)
{
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    char want[8];
    std::snprintf(want, sizeof want, "R%d", ctx->R);
    static const char *kst[] = {"f32", "f16", "bf16"};
    while (std::fgets(line, sizeof line, f)) {
        char ver[8], id[160], rr[8], dt[8];
        long long nx, ny, nz, pitch;
        stencil_tile c = {};
        double a = 0, b = 0;
        int n = std::sscanf(line, "%7s %159s %7s %7s %lld %lld %lld %lld %d %d %d %d %d %d %d %d %lf %lf", ver, id, rr,
                            dt, &nx, &ny, &nz, &pitch, &c.kind, &c.bx, &c.by, &c.ry, &c.dz, &c.vw, &c.xcd, &c.pf, &a,
                            &b);
        if (n != 18) continue;
        if (std::strcmp(ver, "v2") || build_id() != id) continue;
        if (std::strcmp(rr, want) || std::strcmp(dt, kst[ctx->st])) continue;
        if (nx != ctx->d.nx || ny != ctx->d.ny || nz != ctx->d.nz || pitch != ctx->pitch) continue;
        if ((c.kind == STENCIL_TILE_ZMARCH2) != two) continue;
        *t = c;
        *mn = a;
        *act = b;
        found = true;
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const stencil_ctx *ctx, const stencil_tile &t, double mn, double act)
{
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    static const char *kst[] = {"f32", "f16", "bf16"};
    std::fprintf(f, "v2 %s R%d %s %lld %lld %lld %lld %d %d %d %d %d %d %d %d %.6f %.6f\n", build_id().c_str(),
                 ctx->R, kst[ctx->st], (long long)ctx->d.nx, (long long)ctx->d.ny, (long long)ctx->d.nz,
                 (long long)ctx->pitch, t.kind, t.bx, t.by, t.ry, t.dz, t.vw, t.xcd, t.pf, mn, act);
    std::fclose(f);
}

bool overlaps(const void *a, const void *b, int64_t bytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + (uintptr_t)bytes && y < x + (uintptr_t)bytes;
}

// [a, a + la) and [b, b + lb) share a byte.
bool overlaps2(const void *a, int64_t la, const void *b, int64_t lb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + (uintptr_t)lb && y < x + (uintptr_t)la;
}

// Makes ctx->d.device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    hipError_t status = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        status = hipGetDevice(&prev);
        if (status == hipSuccess && prev != dev) status = hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

stencil_status hip_fail(stencil_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, STENCIL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Enqueue one step with a given (already checked) tile.
hipError_t enqueue_step(const stencil_ctx *ctx, const stencil_tile &t, const float *kappa, const void *ucur,
                        const void *uprev, void *unext, int64_t it, const stencil_src *src, hipStream_t s)
{
    const stencil_desc &d = ctx->d;
    SweepArgs a = {};
    a.kappa = kappa;
    a.ucur = ucur;
    a.uprev = uprev;
    a.unext = unext;
    a.nx = (int)d.nx;
    a.pitch = (int)ctx->pitch;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    for (int m = 0; m <= ctx->R; ++m) a.c[m] = ctx->cf[m];
    a.scale = ctx->scale;
    const int nsrc = src ? src->n : 0;
    a.nsrc = (nsrc == 1) ? 1 : 0;
    a.src_idx = nsrc == 1 ? src->idx : nullptr;
    a.src_amp = nsrc == 1 ? src->amp : nullptr;
    a.it = it;
    hipError_t e;
    if (t.kind == STENCIL_TILE_PLAIN) {
        e = p1310::launch_plain(ctx->R, ctx->st, t.bx, t.by, t.dz, a, s);
    } else {
        const ZVariant *v = find_variant(ctx, t);
        if (!v) return hipErrorInvalidValue;
        a.dz = t.dz;
        a.gx = (int)((d.nx + (int64_t)t.bx * t.vw - 1) / ((int64_t)t.bx * t.vw));
        a.gy = (int)((d.ny + (int64_t)t.by * t.ry - 1) / ((int64_t)t.by * t.ry));
        a.gz = (int)((d.nz + t.dz - 1) / t.dz);
        a.xcd = t.xcd;
        e = p1310::launch_zmarch(*v, a, s);
    }
    if (e != hipSuccess) return e;
    if (nsrc > 1)
        e = p1310::launch_inject(ctx->st, unext, kappa, nstore(ctx), ctx->pitch, ctx->d.nx, src->idx, src->amp, nsrc,
                                 it, ctx->scale, s);
    return e;
}

// ---------------------------------------------------------------------------
// Candidate tiles of the search.
// ---------------------------------------------------------------------------
bool same_tile(const stencil_tile &a, const stencil_tile &b)
{
    return a.kind == b.kind && a.bx == b.bx && a.by == b.by && a.ry == b.ry && a.dz == b.dz && a.vw == b.vw &&
           a.xcd == b.xcd && a.pf == b.pf;
}

void push_unique(stencil_ctx *ctx, std::vector<stencil_tile> &out, const stencil_tile &t)
{
    stencil_tile norm;
    std::string keep = ctx->err;
    if (check_tile(ctx, t, &norm) != STENCIL_OK) {
        ctx->err = keep;
        return;
    }
    for (const auto &o : out)
        if (same_tile(o, norm)) return;
    out.push_back(norm);
}

int64_t snap(int64_t v, const std::vector<int64_t> &legal)
{
    int64_t best = legal[0];
    for (int64_t l : legal)
        if (std::llabs(l - v) < std::llabs(best - v)) best = l;
    return best;
}

std::vector<stencil_tile> make_candidates(stencil_ctx *ctx, const stencil_tune_opts &o)
{
    std::vector<stencil_tile> out;
    const stencil_desc &d = ctx->d;
    if (o.temporal == 2) {
        const int vw = vec4_ok(ctx) ? 4 : 1;
        // Two-step shapes x march depths x XCD order. A two-step workgroup
        // covers a large tile, so a grid gives few of them: besides the
        // powers of two, depths that split nz into k equal chunks (k = 2..8)
        // let the search find a workgroup count that fills whole rounds of
        // CUs.
        std::vector<int64_t> dzs = {16, 32, 64, 128, 256, d.nz};
        for (int64_t k = 2; k <= 8; ++k) {
            const int64_t dz = (d.nz + k - 1) / k;
            if (dz >= 16) dzs.push_back(dz);
        }
        for (int i = 0; i < p1310::zmarch2_variant_count(); ++i) {
            const Z2Variant *v = p1310::zmarch2_variant(i);
            if (v->R != ctx->R || v->st != ctx->st || v->vw != vw) continue;
            for (int64_t dz : dzs) {
                if (dz > d.nz) continue;
                for (int xcd = 1; xcd >= 0; --xcd) {
                    stencil_tile t = {STENCIL_TILE_ZMARCH2, v->bx, v->by, 1, (int32_t)dz, v->vw, xcd, v->pf};
                    push_unique(ctx, out, t);
                    // Edge pacing, with the XCD order that lets neighbours
                    // share an L2 (the pause that keeps the edge tiles in
                    // step depends on the plane time: three lengths).
                    for (int pace = 4; xcd && pace <= 6; ++pace) {
                        t.pf = v->pf | (pace << 1);
                        push_unique(ctx, out, t);
                    }
                }
            }
        }
        return out;
    }
    // The widest vector width that divides nx, timed against the next
    // narrower one: two-point against one-point vectors (their rows need not
    // be 16-byte aligned), eight-point (16-bit storage) against four-point.
    const int vw = auto_vw(ctx);
    const int vw_alt = vw == 2 ? 1 : (vw == 8 ? 4 : vw);
    std::vector<const ZVariant *> vars;
    for (int i = 0; i < p1310::zmarch_variant_count(); ++i) {
        const ZVariant *v = p1310::zmarch_variant(i);
        if (v->R == ctx->R && v->st == ctx->st && (v->vw == vw || v->vw == vw_alt)) vars.push_back(v);
    }
    if (zmarch_possible(ctx) && !vars.empty()) {
        if (o.parts < 2) {
            // Every compiled tile shape x a list of z-march depths x XCD order on/off.
            std::vector<int64_t> dzs = {16, 32, 64, 128, 256};
            // Short grids: more, shallower columns keep every CU busy.
            if (d.nz <= 256) dzs.insert(dzs.begin(), 8);
            if (d.nz <= 128) dzs.insert(dzs.begin(), 4);
            dzs.push_back(d.nz);
            for (const ZVariant *v : vars)
                for (int64_t dz : dzs) {
                    if (dz > d.nz) continue;
                    for (int xcd = 1; xcd >= 0; --xcd) {
                        stencil_tile t = {STENCIL_TILE_ZMARCH, v->bx, v->by, v->ry, (int32_t)dz, v->vw, xcd, v->pf};
                        push_unique(ctx, out, t);
                    }
                }
        } else {
            // The paper's P-part grid over the three block extents
            // (tile width, tile height, march depth), each snapped to the
            // nearest extent a compiled kernel provides.
            std::vector<int64_t> ltx, lty;
            for (const ZVariant *v : vars) {
                ltx.push_back((int64_t)v->bx * v->vw);
                lty.push_back((int64_t)v->by * v->ry);
            }
            std::vector<int64_t> bi(o.parts), bj(o.parts), bk(o.parts);
            bi.resize(stencil_pgrid(d.nx, o.parts, bi.data(), o.parts));
            bj.resize(stencil_pgrid(d.ny, o.parts, bj.data(), o.parts));
            bk.resize(stencil_pgrid(d.nz, o.parts, bk.data(), o.parts));
            for (int64_t a : bi)
                for (int64_t b : bj)
                    for (int64_t c : bk) {
                        const int64_t tx = snap(a, ltx), ty = snap(b, lty);
                        for (const ZVariant *v : vars)
                            if ((int64_t)v->bx * v->vw == tx && (int64_t)v->by * v->ry == ty) {
                                stencil_tile t = {STENCIL_TILE_ZMARCH, v->bx, v->by, v->ry, (int32_t)c, v->vw, 1, v->pf};
                                push_unique(ctx, out, t);
                            }
                    }
        }
    }
    if (o.include_plain || out.empty()) {
        const int shapes[][3] = {{64, 4, 1}, {64, 2, 2}, {32, 8, 1}, {128, 2, 1}, {256, 1, 1}, {64, 4, 4}, {32, 4, 8}};
        for (const auto &sh : shapes) {
            stencil_tile t = {STENCIL_TILE_PLAIN, sh[0], sh[1], 1, sh[2], 1, 0, 0};
            push_unique(ctx, out, t);
        }
    }
    return out;
}

// Time `steps` steps of a tile (after `warm` untimed ones) on the stream;
// returns milliseconds, or +inf if a launch failed.
double time_tile(stencil_ctx *ctx, const stencil_tile &t, const float *kappa, void *&a, void *&b, int warm,
                 int steps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, hipError_t *err)
{
    for (int i = 0; i < warm; ++i) {
        hipError_t e = enqueue_step(ctx, t, kappa, a, b, b, 0, nullptr, s);
        if (e != hipSuccess) {
            *err = e;
            return std::numeric_limits<double>::infinity();
        }
        std::swap(a, b);
    }
    hipEventRecord(e0, s);
    for (int i = 0; i < steps; ++i) {
        hipError_t e = enqueue_step(ctx, t, kappa, a, b, b, 0, nullptr, s);
        if (e != hipSuccess) {
            *err = e;
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            return std::numeric_limits<double>::infinity();
        }
        std::swap(a, b);
    }
    hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) {
        *err = e;
        return std::numeric_limits<double>::infinity();
    }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    return ms;
}

// Enqueue one two-step launch (u^{it+1} and u^{it+2}) with a checked tile.
hipError_t enqueue_step2(const stencil_ctx *ctx, const stencil_tile &t, const float *kappa, const void *ucur,
                         const void *uprev, void *unext, void *unext2, int64_t it, const stencil_src *src,
                         hipStream_t s)
{
    const stencil_desc &d = ctx->d;
    const Z2Variant *v = find_variant2(ctx, t);
    if (!v) return hipErrorInvalidValue;
    SweepArgs a = {};
    a.kappa = kappa;
    a.ucur = ucur;
    a.uprev = uprev;
    a.unext = unext;
    a.unext2 = unext2;
    a.nx = (int)d.nx;
    a.pitch = (int)ctx->pitch;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    for (int m = 0; m <= ctx->R; ++m) a.c[m] = ctx->cf[m];
    a.scale = ctx->scale;
    a.nsrc = (src && src->n == 1) ? 1 : 0;
    a.src_idx = a.nsrc ? src->idx : nullptr;
    a.src_amp = a.nsrc ? src->amp : nullptr;
    a.it = it;
    a.dz = t.dz;
    a.gx = (int)((d.nx + v->own_x - 1) / v->own_x);
    a.gy = (int)((d.ny + v->own_y - 1) / v->own_y);
    a.gz = (int)((d.nz + t.dz - 1) / t.dz);
    a.xcd = t.xcd;
    a.pace = (t.pf >> 1) & 7;
    return p1310::launch_zmarch2(*v, a, s);
}

// Time `steps` steps (steps/2 two-step launches, steps even) of a two-step
// tile over four scratch fields; +inf if a launch failed.
double time_tile2(stencil_ctx *ctx, const stencil_tile &t, const float *kappa, void *f[4], int warm, int steps,
                  hipStream_t s, hipEvent_t e0, hipEvent_t e1, hipError_t *err)
{
    auto launch = [&]() -> hipError_t {
        hipError_t e = enqueue_step2(ctx, t, kappa, f[0], f[1], f[2], f[3], 0, nullptr, s);
        // (u^{n+2}, u^{n+1}) become the inputs; the old inputs are free.
        void *cur = f[0], *prev = f[1];
        f[0] = f[3];
        f[1] = f[2];
        f[2] = prev;
        f[3] = cur;
        return e;
    };
    for (int i = 0; i < (warm + 1) / 2; ++i) {
        hipError_t e = launch();
        if (e != hipSuccess) {
            *err = e;
            return std::numeric_limits<double>::infinity();
        }
    }
    hipEventRecord(e0, s);
    for (int i = 0; i < steps / 2; ++i) {
        hipError_t e = launch();
        if (e != hipSuccess) {
            *err = e;
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            return std::numeric_limits<double>::infinity();
        }
    }
    hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) {
        *err = e;
        return std::numeric_limits<double>::infinity();
    }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    return ms;
}

}  // namespace

extern "C" {

const char *stencil_strerror(stencil_status s)
{
    switch (s) {
    case STENCIL_OK: return "success";
    case STENCIL_EINVAL: return "invalid argument";
    case STENCIL_EUNSTABLE: return "time step above the leapfrog stability limit";
    case STENCIL_ENOMEM: return "out of host memory";
    case STENCIL_EDEVICE: return "HIP device error";
    case STENCIL_EUNSUPPORTED: return "unsupported storage type or tile";
    case STENCIL_EALIAS: return "u_cur and u_prev_next overlap";
    case STENCIL_EDIVERGED: return "the wavefield diverged (not finite or above the limit)";
    }
    return "unknown status";
}

const char *stencil_last_error(const stencil_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

const char *stencil_build_id(void) { return build_id().c_str(); }

double stencil_cfl_limit(int32_t radius) { return radius_ok(radius) ? cfl_limit_of(radius) : -1.0; }

int32_t stencil_coefficients(int32_t radius, float *out)
{
    if (!radius_ok(radius) || !out) return STENCIL_EINVAL;
    Rat c[p1310::kMaxRadius + 1];
    weights(radius, c);
    out[0] = (float)rat_to_double(rmul(c[0], 3));
    for (int m = 1; m <= radius; ++m) out[m] = (float)rat_to_double(c[m]);
    return radius + 1;
}

stencil_status stencil_init(const stencil_desc *d, stencil_ctx **out)
{
    if (!d || !out) return STENCIL_EINVAL;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 0x7fffffff || d->ny > 0x7fffffff || d->nz > 0x7fffffff)
        return STENCIL_EINVAL;
    if (d->pitch != 0 && (d->pitch < d->nx || d->pitch > 0x7fffffff)) return STENCIL_EINVAL;
    const int64_t pitch = d->pitch ? d->pitch : d->nx;
    if (pitch * d->ny > ((int64_t)1 << 29)) return STENCIL_EINVAL;  // plane byte offsets are 32-bit
    if (!radius_ok(d->radius)) return STENCIL_EINVAL;
    if (d->storage != STENCIL_F32 && d->storage != STENCIL_F16 && d->storage != STENCIL_BF16)
        return STENCIL_EUNSUPPORTED;
    if (d->storage != STENCIL_F32 && d->radius < 4) return STENCIL_EUNSUPPORTED;  // 16-bit kernels: R = 4, 5
    const double scale = d->storage_scale == 0.0 ? 1.0 : d->storage_scale;
    {
        int ex = 0;
        if (!(scale > 0) || !std::isfinite(scale) || std::frexp(scale, &ex) != 0.5 || ex < -100 || ex > 100)
            return STENCIL_EINVAL;  // a power of two, so scaling is exact
    }
    if (!(d->h > 0) || !(d->dt > 0) || !(d->vmax > 0) || !std::isfinite(d->h) || !std::isfinite(d->dt) ||
        !std::isfinite(d->vmax))
        return STENCIL_EINVAL;
    if (d->device < 0) return STENCIL_EINVAL;
    if (d->vmax * d->dt / d->h > cfl_limit_of(d->radius)) return STENCIL_EUNSTABLE;
    stencil_ctx *ctx = new (std::nothrow) stencil_ctx;
    if (!ctx) return STENCIL_ENOMEM;
    ctx->d = *d;
    ctx->pitch = pitch;
    ctx->R = d->radius;
    ctx->st = d->storage;
    ctx->es = d->storage == STENCIL_F32 ? 4 : 2;
    ctx->scale = (float)scale;
    stencil_coefficients(ctx->R, ctx->cf);
    stencil_tile t = default_tile(ctx);
    const char *origin = "default";
    if (d->tile.kind != STENCIL_TILE_AUTO) {
        t = d->tile;
        origin = "given";
    } else {
        double mn, act;
        stencil_tile c;
        if (cache_lookup(std::getenv("STENCIL_TUNE_CACHE"), ctx, false, &c, &mn, &act)) {
            t = c;
            origin = "tune cache";
        }
    }
    stencil_tile norm;
    stencil_status st = check_tile(ctx, t, &norm);
    if (st != STENCIL_OK && d->tile.kind == STENCIL_TILE_AUTO) {
        st = check_tile(ctx, default_tile(ctx), &norm);  // bad cache entry: fall back
        origin = "default (the tune cache entry is not runnable)";
    }
    if (st != STENCIL_OK) {
        delete ctx;
        return st;
    }
    ctx->tile = norm;
    if (check_tile(ctx, default_tile2(ctx), &norm) == STENCIL_OK) ctx->tile2 = norm;
    ctx->err.clear();
    if (log_on())
        std::fprintf(stderr, "stencil: init %lldx%lldx%lld R%d %s device %d, tile %s (%s)\n", (long long)d->nx,
                     (long long)d->ny, (long long)d->nz, ctx->R, storage_name(ctx->st), d->device,
                     tile_text(ctx->tile).c_str(), origin);
    *out = ctx;
    return STENCIL_OK;
}

void stencil_destroy(stencil_ctx *ctx) { delete ctx; }

stencil_status stencil_get_tile(const stencil_ctx *ctx, stencil_tile *out)
{
    if (!ctx || !out) return STENCIL_EINVAL;
    *out = ctx->tile;
    return STENCIL_OK;
}

stencil_status stencil_set_tile(stencil_ctx *ctx, const stencil_tile *tile)
{
    if (!ctx || !tile) return STENCIL_EINVAL;
    stencil_tile norm;
    stencil_tile t = *tile;
    if (t.kind == STENCIL_TILE_AUTO) t = default_tile(ctx);
    stencil_status st = check_tile(ctx, t, &norm);
    if (st != STENCIL_OK) return st;
    if (norm.kind == STENCIL_TILE_ZMARCH2) ctx->tile2 = norm;
    else ctx->tile = norm;
    return STENCIL_OK;
}

stencil_status stencil_get_tile2(const stencil_ctx *ctx, stencil_tile *out)
{
    if (!ctx || !out) return STENCIL_EINVAL;
    if (ctx->tile2.kind != STENCIL_TILE_ZMARCH2) return STENCIL_EUNSUPPORTED;
    *out = ctx->tile2;
    return STENCIL_OK;
}

int32_t stencil_list_tiles2(int32_t radius, int32_t vec4, stencil_tile *out, int32_t cap)
{
    if (!radius_ok(radius) || cap < 0) return STENCIL_EINVAL;
    int32_t n = 0;
    for (int i = 0; i < p1310::zmarch2_variant_count(); ++i) {
        const Z2Variant *v = p1310::zmarch2_variant(i);
        if (v->R != radius || v->vw != (vec4 ? 4 : 1)) continue;
        if (out && n < cap) {
            stencil_tile t = {};
            t.kind = STENCIL_TILE_ZMARCH2;
            t.bx = v->bx;
            t.by = v->by;
            t.ry = 1;
            t.vw = v->vw;
            t.pf = v->pf;
            out[n] = t;
        }
        ++n;
    }
    return n;
}

stencil_status stencil_step2(stencil_ctx *ctx, const void *kappa, const void *u_cur, const void *u_prev,
                             void *u_next, void *u_next2, int64_t it, const stencil_src *src, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!kappa || !u_cur || !u_prev || !u_next || !u_next2) return fail(ctx, STENCIL_EINVAL, "null field pointer");
    if (ctx->tile2.kind != STENCIL_TILE_ZMARCH2)
        return fail(ctx, STENCIL_EUNSUPPORTED, "no two-step kernel for this radius and storage");
    const int64_t ub = nstore(ctx) * ctx->es, kb = nstore(ctx) * 4;
    const void *f[] = {u_cur, u_prev, u_next, u_next2};
    for (int i = 0; i < 4; ++i) {
        if (overlaps2(kappa, kb, f[i], ub)) return fail(ctx, STENCIL_EALIAS, "kappa overlaps a wavefield");
        for (int j = i + 1; j < 4; ++j)
            if (overlaps(f[i], f[j], ub)) return fail(ctx, STENCIL_EALIAS, "the four wavefields must not overlap");
    }
    if (!vec_aligned(ctx, ctx->tile2.vw, kappa, {u_cur, u_prev, u_next, u_next2}))
        return fail(ctx, STENCIL_EINVAL, "kappa must be 4*vw-byte and the wavefields vw-value aligned");
    if (src && src->n != 0) {
        if (src->n < 0) return fail(ctx, STENCIL_EINVAL, "bad source description");
        if (src->n > 1) return fail(ctx, STENCIL_EUNSUPPORTED, "two-step launches take at most one source");
        if (!src->idx || !src->amp) return fail(ctx, STENCIL_EINVAL, "bad source description");
        if (it < 0 || it + 1 >= src->nt) return fail(ctx, STENCIL_EINVAL, "steps it and it+1 need source samples");
    }
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = enqueue_step2(ctx, ctx->tile2, (const float *)kappa, u_cur, u_prev, u_next, u_next2, it,
                                 (src && src->n) ? src : nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "two-step sweep launch");
    return STENCIL_OK;
}

int32_t stencil_list_tiles(int32_t radius, int32_t vec4, int32_t storage, stencil_tile *out, int32_t cap)
{
    if (!radius_ok(radius) || cap < 0 || storage < STENCIL_F32 || storage > STENCIL_BF16) return STENCIL_EINVAL;
    int32_t n = 0;
    for (int i = 0; i < p1310::zmarch_variant_count(); ++i) {
        const ZVariant *v = p1310::zmarch_variant(i);
        if (v->R != radius || v->st != storage || v->vw != (vec4 == 2 || vec4 == 8 ? vec4 : (vec4 ? 4 : 1))) continue;
        if (out && n < cap) {
            stencil_tile t = {};
            t.kind = STENCIL_TILE_ZMARCH;
            t.bx = v->bx;
            t.by = v->by;
            t.ry = v->ry;
            t.vw = v->vw;
            t.pf = v->pf;
            out[n] = t;
        }
        ++n;
    }
    return n;
}

stencil_status stencil_kappa(stencil_ctx *ctx, const void *v, void *kappa, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!v || !kappa) return fail(ctx, STENCIL_EINVAL, "null pointer");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = p1310::launch_kappa((const float *)v, (float *)kappa, nstore(ctx), ctx->d.dt, ctx->d.h,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kappa launch");
    return STENCIL_OK;
}

stencil_status stencil_step_to(stencil_ctx *ctx, const void *kappa, const void *u_cur, const void *u_prev,
                               void *u_next, int64_t it, const stencil_src *src, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!kappa || !u_cur || !u_prev || !u_next) return fail(ctx, STENCIL_EINVAL, "null field pointer");
    const int64_t bytes = nstore(ctx) * ctx->es, kbytes = nstore(ctx) * 4;
    if (overlaps(u_cur, u_next, bytes)) return fail(ctx, STENCIL_EALIAS, "u_cur overlaps the output");
    if (overlaps2(kappa, kbytes, u_next, bytes)) return fail(ctx, STENCIL_EALIAS, "kappa overlaps the output");
    if (u_prev != u_next && overlaps(u_prev, u_next, bytes))
        return fail(ctx, STENCIL_EALIAS, "u_prev partially overlaps the output");
    if (ctx->tile.kind == STENCIL_TILE_ZMARCH && !vec_aligned(ctx, ctx->tile.vw, kappa, {u_cur, u_prev, u_next}))
        return fail(ctx, STENCIL_EINVAL, "kappa must be 4*vw-byte and the wavefields vw-value aligned");
    if (src && src->n != 0) {
        if (src->n < 0 || !src->idx || !src->amp) return fail(ctx, STENCIL_EINVAL, "bad source description");
        if (it < 0 || it >= src->nt) return fail(ctx, STENCIL_EINVAL, "step index outside the source's samples");
    }
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = enqueue_step(ctx, ctx->tile, (const float *)kappa, (const float *)u_cur, (const float *)u_prev,
                                (float *)u_next, it, (src && src->n) ? src : nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "sweep launch");
    return STENCIL_OK;
}

stencil_status stencil_step(stencil_ctx *ctx, const void *kappa, const void *u_cur, void *u_prev_next, int64_t it,
                            const stencil_src *src, void *stream)
{
    return stencil_step_to(ctx, kappa, u_cur, u_prev_next, u_prev_next, it, src, stream);
}

stencil_status stencil_select(const double *t, int32_t n_nodes, int32_t n_cores, int32_t n_cand, int32_t policy,
                              int32_t *best_id, double *best_time)
{
    if (!t || !best_id || !best_time || n_nodes < 1 || n_cores < 1 || n_cand < 1) return STENCIL_EINVAL;
    if (policy < STENCIL_POLICY_WORST || policy > STENCIL_POLICY_OB) return STENCIL_EINVAL;
    auto at = [&](int i, int k, int j) { return t[((int64_t)i * n_cores + k) * n_cand + j]; };
    if (policy == STENCIL_POLICY_OB) {
        int bi = 0, bj = 0;
        double bt = at(0, 0, 0);
        for (int i = 0; i < n_nodes; ++i)
            for (int k = 0; k < n_cores; ++k)
                for (int j = 0; j < n_cand; ++j)
                    if (at(i, k, j) < bt) {
                        bt = at(i, k, j);
                        bi = i;
                        bj = j;
                    }
        *best_id = bi * n_cand + bj;
        *best_time = bt;
        return STENCIL_OK;
    }
    double node_t = 0;
    int node_id = -1;
    std::vector<int> win(n_cores);
    std::vector<double> wt(n_cores);
    for (int i = 0; i < n_nodes; ++i) {
        // Stage 1: every core keeps its fastest candidate (first on ties).
        for (int k = 0; k < n_cores; ++k) {
            int bj = 0;
            for (int j = 1; j < n_cand; ++j)
                if (at(i, k, j) < at(i, k, bj)) bj = j;
            win[k] = bj;
            wt[k] = at(i, k, bj);
        }
        // Stage 2: one core winner per node by the policy (first core on ties).
        int pick = 0;
        if (policy == STENCIL_POLICY_MIN) {
            for (int k = 1; k < n_cores; ++k)
                if (wt[k] < wt[pick]) pick = k;
        } else if (policy == STENCIL_POLICY_WORST) {
            for (int k = 1; k < n_cores; ++k)
                if (wt[k] > wt[pick]) pick = k;
        } else {
            double mean = 0;
            for (int k = 0; k < n_cores; ++k) mean += wt[k];
            mean /= n_cores;
            for (int k = 1; k < n_cores; ++k)
                if (std::fabs(wt[k] - mean) < std::fabs(wt[pick] - mean)) pick = k;
        }
        // Stage 3: the fastest node choice (first node on ties).
        if (node_id < 0 || wt[pick] < node_t) {
            node_t = wt[pick];
            node_id = i * n_cand + win[pick];
        }
    }
    *best_id = node_id;
    *best_time = node_t;
    return STENCIL_OK;
}

int32_t stencil_pgrid(int64_t S, int32_t P, int64_t *out, int32_t cap)
{
    if (S < 1 || P < 2 || cap < 0) return STENCIL_EINVAL;
    int32_t n = 0;
    int64_t last = -1;
    for (int64_t j = 0; j < P; ++j) {
        int64_t b = 1 + (j * S) / (P - 1);
        if (b > S) b = S;
        if (b == last) continue;
        last = b;
        if (out && n < cap) out[n] = b;
        ++n;
    }
    return n;
}


stencil_status stencil_tune(stencil_ctx *ctx, const void *kappa, void *scratch_a, void *scratch_b,
                            const stencil_tune_opts *opts, stencil_tune_report *report, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!kappa || !scratch_a || !scratch_b || !report) return fail(ctx, STENCIL_EINVAL, "null pointer");
    const int64_t bytes = nstore(ctx) * ctx->es, kbytes = nstore(ctx) * 4;
    if (overlaps(scratch_a, scratch_b, bytes) || overlaps2(kappa, kbytes, scratch_a, bytes) ||
        overlaps2(kappa, kbytes, scratch_b, bytes))
        return fail(ctx, STENCIL_EALIAS, "kappa and the two scratch fields must not overlap");
    if (((uintptr_t)kappa | (uintptr_t)scratch_a | (uintptr_t)scratch_b) & 15u)
        return fail(ctx, STENCIL_EINVAL, "fields must be 16-byte aligned");
    stencil_tune_opts o = {};
    if (opts) o = *opts;
    if (o.policy < STENCIL_POLICY_WORST || o.policy > STENCIL_POLICY_OB) return fail(ctx, STENCIL_EINVAL, "bad policy");
    if (o.n_iter < 0 || o.n_rep < 0 || o.parts < 0 || o.parts == 1 || o.table_cap < 0 ||
        (o.temporal != 0 && o.temporal != 1 && o.temporal != 2))
        return fail(ctx, STENCIL_EINVAL, "bad tune options");
    const bool two = o.temporal == 2;
    if (two) {
        if (ctx->tile2.kind != STENCIL_TILE_ZMARCH2)
            return fail(ctx, STENCIL_EUNSUPPORTED, "no two-step kernel for this radius and storage");
        if (!o.scratch_c || !o.scratch_d) return fail(ctx, STENCIL_EINVAL, "two-step search needs scratch_c and scratch_d");
        const void *f[] = {scratch_a, scratch_b, o.scratch_c, o.scratch_d};
        for (int i = 0; i < 4; ++i) {
            if (overlaps2(kappa, kbytes, f[i], bytes) || (((uintptr_t)f[i]) & 15u))
                return fail(ctx, overlaps2(kappa, kbytes, f[i], bytes) ? STENCIL_EALIAS : STENCIL_EINVAL,
                            "bad scratch field");
            for (int j = i + 1; j < 4; ++j)
                if (overlaps(f[i], f[j], bytes)) return fail(ctx, STENCIL_EALIAS, "scratch fields overlap");
        }
    }
    int n_iter = o.n_iter ? o.n_iter : 10;
    if (two && (n_iter & 1)) ++n_iter;
    const int n_rep = o.n_rep ? o.n_rep : 3;
    const int warm = o.warmup == 0 ? 2 : (o.warmup < 0 ? 0 : o.warmup);
    *report = stencil_tune_report{};
    const auto t_start = std::chrono::steady_clock::now();

    {
        stencil_tile c;
        double mn, act;
        if (cache_lookup(o.cache_path, ctx, two, &c, &mn, &act)) {
            stencil_tile norm;
            if (check_tile(ctx, c, &norm) == STENCIL_OK) {
                if (two) ctx->tile2 = norm;
                else ctx->tile = norm;
                report->tile = norm;
                report->min_time_ms = mn;
                report->actual_time_ms = act;
                report->gap = (act - mn) / mn;
                report->from_cache = 1;
                report->n_candidates = 0;
                if (log_on())
                    std::fprintf(stderr, "stencil: tune %lldx%lldx%lld R%d %s: from the cache %s: %s\n",
                                 (long long)ctx->d.nx, (long long)ctx->d.ny, (long long)ctx->d.nz, ctx->R,
                                 storage_name(ctx->st), o.cache_path, tile_text(norm).c_str());
                return STENCIL_OK;
            }
        }
    }

    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    std::vector<stencil_tile> cands = make_candidates(ctx, o);
    const int nC = (int)cands.size();
    if (nC == 0) return fail(ctx, STENCIL_EUNSUPPORTED, "no candidate tile fits this grid");
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipEventCreate");
    he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(ctx, he, "hipEventCreate");
    }
    void *a = scratch_a, *b = scratch_b;
    void *f4[4] = {scratch_a, scratch_b, o.scratch_c, o.scratch_d};
    const float *k = (const float *)kappa;
    auto time_any = [&](const stencil_tile &t, hipError_t *e) {
        return two ? time_tile2(ctx, t, k, f4, warm, n_iter, s, e0, e1, e)
                   : time_tile(ctx, t, k, a, b, warm, n_iter, s, e0, e1, e);
    };
    std::vector<double> table((size_t)n_rep * nC, std::numeric_limits<double>::infinity());
    hipError_t last = hipSuccess;

    // Selection phase: every replicate times every candidate in the same order.
    for (int r = 0; r < n_rep; ++r)
        for (int c = 0; c < nC; ++c) {
            hipError_t e = hipSuccess;
            table[(size_t)r * nC + c] = time_any(cands[c], &e);
            if (e != hipSuccess) last = e;
        }
    bool any = false;
    for (double v : table) any = any || std::isfinite(v);
    if (!any) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return hip_fail(ctx, last == hipSuccess ? hipErrorLaunchFailure : last, "every candidate failed");
    }
    int32_t best = 0;
    double min_time = 0;
    stencil_select(table.data(), 1, n_rep, nC, o.policy, &best, &min_time);

    // Verification phase: the chosen tile again, then the default for context.
    hipError_t e = hipSuccess;
    const double actual = time_any(cands[best], &e);
    stencil_tile dflt;
    double dtime = std::numeric_limits<double>::infinity();
    if (check_tile(ctx, two ? default_tile2(ctx) : default_tile(ctx), &dflt) == STENCIL_OK) dtime = time_any(dflt, &e);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!std::isfinite(actual)) return hip_fail(ctx, e, "verification run failed");

    if (two) ctx->tile2 = cands[best];
    else ctx->tile = cands[best];
    report->tile = cands[best];
    report->min_time_ms = min_time;
    report->actual_time_ms = actual;
    report->gap = (actual - min_time) / min_time;
    report->default_time_ms = dtime;
    report->n_candidates = nC;
    report->from_cache = 0;
    report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (o.table && o.table_cap > 0)
        for (int r = 0; r < n_rep; ++r)
            for (int c = 0; c < nC && c < o.table_cap; ++c) o.table[(size_t)r * o.table_cap + c] = table[(size_t)r * nC + c];
    if (o.candidates)
        for (int c = 0; c < nC && c < o.table_cap; ++c) o.candidates[c] = cands[c];
    cache_store(o.cache_path, ctx, cands[best], min_time, actual);
    if (log_on())
        std::fprintf(stderr,
                     "stencil: tune %lldx%lldx%lld R%d %s%s: %d candidates x %d replicates x %d steps, chose %s, "
                     "MinTime %.4f ms, ActualTime %.4f ms, gap %+.2f%%, default tile %.4f ms, %.2f s\n",
                     (long long)ctx->d.nx, (long long)ctx->d.ny, (long long)ctx->d.nz, ctx->R, storage_name(ctx->st),
                     two ? " two-step" : "", nC, n_rep, n_iter, tile_text(cands[best]).c_str(), min_time, actual,
                     100.0 * report->gap, dtime, report->seconds);
    return STENCIL_OK;
}

stencil_status stencil_kappa_slowness2(stencil_ctx *ctx, const void *m, void *kappa, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!m || !kappa) return fail(ctx, STENCIL_EINVAL, "null pointer");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = p1310::launch_kappa_m((const float *)m, (float *)kappa, nstore(ctx), ctx->d.dt, ctx->d.h,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kappa launch");
    return STENCIL_OK;
}

stencil_status stencil_sample(stencil_ctx *ctx, const void *u, const int64_t *idx, int32_t n, void *out,
                              void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (ctx->st != p1310::kF32) return fail(ctx, STENCIL_EUNSUPPORTED, "receiver samples need FP32 storage");
    if (n < 0) return fail(ctx, STENCIL_EINVAL, "negative receiver count");
    if (n == 0) return STENCIL_OK;
    if (!u || !idx || !out) return fail(ctx, STENCIL_EINVAL, "null pointer");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = p1310::launch_sample((const float *)u, nstore(ctx), ctx->pitch, ctx->d.nx, idx, n, (float *)out,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "sample launch");
    return STENCIL_OK;
}

stencil_status stencil_adjoint_step(stencil_ctx *ctx, const void *kappa, const void *lam_cur, void *lam_prev_next,
                                    int64_t it, const stencil_src *resid, const void *u_next, const void *u_cur,
                                    const void *u_prev, double *grad, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (ctx->st != p1310::kF32) return fail(ctx, STENCIL_EUNSUPPORTED, "the adjoint needs FP32 storage");
    if (grad && (!u_next || !u_cur || !u_prev))
        return fail(ctx, STENCIL_EINVAL, "gradient accumulation needs u_next, u_cur and u_prev");
    if (grad) {
        const int64_t fb = nstore(ctx) * 4, gb = nstore(ctx) * 8;
        const void *fields[] = {kappa, lam_cur, lam_prev_next, u_next, u_cur, u_prev};
        for (const void *f : fields)
            if (overlaps2(grad, gb, f, fb)) return fail(ctx, STENCIL_EALIAS, "grad overlaps another field");
        if (overlaps(lam_prev_next, u_next, fb) || overlaps(lam_prev_next, u_cur, fb) ||
            overlaps(lam_prev_next, u_prev, fb))
            return fail(ctx, STENCIL_EALIAS, "lam_prev_next overlaps a forward wavefield");
    }
    // The adjoint variable is mu = kappa * lambda; its recurrence is the
    // forward step with the residuals injected at the receivers.
    stencil_status st = stencil_step(ctx, kappa, lam_cur, lam_prev_next, it, resid, stream);
    if (st != STENCIL_OK || !grad) return st;
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    const double scale = -(ctx->d.h * ctx->d.h) / (ctx->d.dt * ctx->d.dt);
    hipError_t e = p1310::launch_grad(grad, (const float *)lam_prev_next, (const float *)u_next, (const float *)u_cur,
                                      (const float *)u_prev, nstore(ctx), scale, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "gradient launch");
    return STENCIL_OK;
}

stencil_status stencil_gradient2(stencil_ctx *ctx, const void *mu_k, const void *mu_km1, const void *u_k,
                                 const void *u_km1, const void *u_km2, const void *u_km3, double *grad, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (ctx->st != p1310::kF32) return fail(ctx, STENCIL_EUNSUPPORTED, "the gradient needs FP32 storage");
    if (!mu_k || !mu_km1 || !u_k || !u_km1 || !u_km2 || !u_km3 || !grad)
        return fail(ctx, STENCIL_EINVAL, "null pointer");
    const int64_t fb = nstore(ctx) * 4, gb = nstore(ctx) * 8;
    const void *fields[] = {mu_k, mu_km1, u_k, u_km1, u_km2, u_km3};
    for (const void *f : fields)
        if (overlaps2(grad, gb, f, fb)) return fail(ctx, STENCIL_EALIAS, "grad overlaps another field");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    const double scale = -(ctx->d.h * ctx->d.h) / (ctx->d.dt * ctx->d.dt);
    const float *mu[] = {(const float *)mu_k, (const float *)mu_km1};
    const float *u[] = {(const float *)u_k, (const float *)u_km1, (const float *)u_km2, (const float *)u_km3};
    hipError_t e = p1310::launch_gradn(2, grad, mu, u, nstore(ctx), scale, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "gradient launch");
    return STENCIL_OK;
}

stencil_status stencil_gradient_terms(stencil_ctx *ctx, int32_t m, const void *const *mu, const void *const *u,
                                      double *grad, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (ctx->st != p1310::kF32) return fail(ctx, STENCIL_EUNSUPPORTED, "the gradient needs FP32 storage");
    if (m < 1 || m > 4) return fail(ctx, STENCIL_EINVAL, "m must be 1..4");
    if (!mu || !u || !grad) return fail(ctx, STENCIL_EINVAL, "null pointer");
    const int64_t fb = nstore(ctx) * 4, gb = nstore(ctx) * 8;
    const float *fm[4], *fu[6];
    for (int j = 0; j < m; ++j) {
        if (!mu[j]) return fail(ctx, STENCIL_EINVAL, "null pointer");
        if (overlaps2(grad, gb, mu[j], fb)) return fail(ctx, STENCIL_EALIAS, "grad overlaps another field");
        fm[j] = (const float *)mu[j];
    }
    for (int j = 0; j < m + 2; ++j) {
        if (!u[j]) return fail(ctx, STENCIL_EINVAL, "null pointer");
        if (overlaps2(grad, gb, u[j], fb)) return fail(ctx, STENCIL_EALIAS, "grad overlaps another field");
        fu[j] = (const float *)u[j];
    }
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    const double scale = -(ctx->d.h * ctx->d.h) / (ctx->d.dt * ctx->d.dt);
    hipError_t e = p1310::launch_gradn(m, grad, fm, fu, nstore(ctx), scale, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "gradient launch");
    return STENCIL_OK;
}

stencil_status stencil_misfit(const void *traces, const void *observed, int64_t count, void *resid, double *misfit,
                              void *stream)
{
    if (!misfit || count < 0) return STENCIL_EINVAL;
    if (count > 0 && (!traces || !observed)) return STENCIL_EINVAL;  // count 0: J = 0, no sample is read
    hipError_t e = p1310::launch_misfit((const float *)traces, (const float *)observed, count, (float *)resid, misfit,
                                        (hipStream_t)stream);
    return e == hipSuccess ? STENCIL_OK : STENCIL_EDEVICE;
}

// ---------------------------------------------------------------------------
// Static batch table: device memory that stencil_batch_create_static uses for
// the batch kernel's descriptor table instead of a hipMalloc'd one. Each GPU
// holds its own copy of the array at its own address, which
// hipGetSymbolAddress returns with that GPU current (the array's name in host
// code is not a device address). Every static batch on a device shares the
// array; a later stencil_batch_create_static on the device replaces the
// contents, and batches built before it are refused from then on (their
// generation no longer matches).
// ---------------------------------------------------------------------------
constexpr size_t kStaticTableBytes = 64 * 1024;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticTableBytes];

namespace {

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
uint64_t g_static_gen[kMaxDevices] = {};

// Device address of this device's static table (the device must be current).
hipError_t static_table(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_ptr[device] = p;
    }
    *ptr = g_static_ptr[device];
    return hipSuccess;
}

// Builds a batch; tiles[i] (when tiles != NULL) replaces shot i's context tile.
// in_static: the device table goes into the device's static table.
stencil_status build_batch(const stencil_shot *shots, int32_t n, const stencil_tile *tiles, int64_t it0,
                           stencil_batch **out, bool in_static = false)
{
    if (!shots || !out || n < 1 || n > 4096) return STENCIL_EINVAL;
    stencil_batch *bt = new (std::nothrow) stencil_batch;
    if (!bt) return STENCIL_ENOMEM;
    bt->it0 = it0;
    bt->nt_min = std::numeric_limits<int64_t>::max();
    bt->device = shots[0].ctx ? shots[0].ctx->d.device : 0;
    for (int i = 0; i < n; ++i) {
        const stencil_shot &sh = shots[i];
        if (!sh.ctx || !sh.kappa || !sh.u_a || !sh.u_b || sh.ctx->d.device != bt->device) {
            delete bt;
            return STENCIL_EINVAL;
        }
        const int64_t ub = nstore(sh.ctx) * sh.ctx->es, kb = nstore(sh.ctx) * 4;
        if (overlaps(sh.u_a, sh.u_b, ub) || overlaps2(sh.kappa, kb, sh.u_a, ub) || overlaps2(sh.kappa, kb, sh.u_b, ub)) {
            delete bt;
            return STENCIL_EALIAS;
        }
        const stencil_tile &tt = tiles ? tiles[i] : sh.ctx->tile;
        if (tt.kind == STENCIL_TILE_ZMARCH && !vec_aligned(sh.ctx, tt.vw, sh.kappa, {sh.u_a, sh.u_b})) {
            delete bt;
            return STENCIL_EINVAL;
        }
        if (sh.src.n < 0 || (sh.src.n > 0 && (!sh.src.idx || !sh.src.amp || sh.src.nt < 1))) {
            delete bt;
            return STENCIL_EINVAL;
        }
        // One launch sweeps every shot: a buffer that one shot writes must not
        // overlap any field of another (kappa may be shared: it is only read).
        for (int j = 0; j < i; ++j) {
            const stencil_shot &o = shots[j];
            const int64_t oub = nstore(o.ctx) * o.ctx->es, okb = nstore(o.ctx) * 4;
            const void *mine[] = {sh.u_a, sh.u_b}, *theirs[] = {o.u_a, o.u_b};
            bool clash = false;
            for (const void *w : mine)
                clash = clash || overlaps2(w, ub, o.u_a, oub) || overlaps2(w, ub, o.u_b, oub) ||
                        overlaps2(w, ub, o.kappa, okb);
            for (const void *w : theirs) clash = clash || overlaps2(w, oub, sh.kappa, kb);
            if (clash) {
                delete bt;
                return STENCIL_EALIAS;
            }
        }
        if (sh.src.n > 0) bt->nt_min = std::min(bt->nt_min, sh.src.nt);
        bt->shots.push_back({sh.ctx, (const float *)sh.kappa, sh.u_a, sh.u_b, sh.src,
                             tiles ? tiles[i] : sh.ctx->tile});
    }
    // Group the z-march shots by compiled kernel (tile shape) and XCD order.
    for (int i = 0; i < n; ++i) {
        const stencil_tile &t = bt->shots[i].tile;
        if (t.kind != STENCIL_TILE_ZMARCH) {
            bt->solo.push_back(i);
            continue;
        }
        const ZVariant *v = find_variant(bt->shots[i].ctx, t);
        bool placed = false;
        for (auto &g : bt->groups)
            if (g.v == v && g.xcd == t.xcd) {
                ++g.nshots;
                placed = true;
            }
        if (!placed) bt->groups.push_back({v, t.xcd, 1, 0, {nullptr, nullptr}, nullptr});
    }
    // Host tables, then one device allocation for every group.
    std::vector<std::vector<SweepArgs>> tabs[2];
    std::vector<std::vector<int>> begins;
    size_t total = 0;
    for (auto &g : bt->groups) {
        std::vector<SweepArgs> t0, t1;
        std::vector<int> beg;
        int64_t blocks = 0;
        for (int i = 0; i < n; ++i) {
            const auto &sh = bt->shots[i];
            if (sh.tile.kind != STENCIL_TILE_ZMARCH || find_variant(sh.ctx, sh.tile) != g.v || sh.tile.xcd != g.xcd)
                continue;
            const stencil_desc &d = sh.ctx->d;
            SweepArgs a = {};
            a.kappa = sh.kappa;
            a.nx = (int)d.nx;
            a.pitch = (int)sh.ctx->pitch;
            a.ny = (int)d.ny;
            a.nz = (int)d.nz;
            for (int m = 0; m <= sh.ctx->R; ++m) a.c[m] = sh.ctx->cf[m];
            a.scale = sh.ctx->scale;
            a.dz = sh.tile.dz;
            a.gx = (int)((d.nx + (int64_t)sh.tile.bx * sh.tile.vw - 1) / ((int64_t)sh.tile.bx * sh.tile.vw));
            a.gy = (int)((d.ny + (int64_t)sh.tile.by * sh.tile.ry - 1) / ((int64_t)sh.tile.by * sh.tile.ry));
            a.gz = (int)((d.nz + sh.tile.dz - 1) / sh.tile.dz);
            a.xcd = 0;  // the batch applies the XCD order over the whole launch
            a.nsrc = sh.src.n == 1 ? 1 : 0;
            a.src_idx = sh.src.n == 1 ? sh.src.idx : nullptr;
            a.src_amp = sh.src.n == 1 ? sh.src.amp : nullptr;
            beg.push_back((int)blocks);
            blocks += (int64_t)a.gx * a.gy * a.gz;
            SweepArgs e = a, o = a;
            e.ucur = sh.u_a;
            e.uprev = sh.u_b;
            e.unext = sh.u_b;
            o.ucur = sh.u_b;
            o.uprev = sh.u_a;
            o.unext = sh.u_a;
            t0.push_back(e);
            t1.push_back(o);
        }
        if (!launch_fits(blocks, g.v->threads)) {
            delete bt;
            return STENCIL_EUNSUPPORTED;
        }
        g.blocks = (int)blocks;
        tabs[0].push_back(t0);
        tabs[1].push_back(t1);
        begins.push_back(beg);
        total += 2 * round256(t0.size() * sizeof(SweepArgs)) + round256(beg.size() * sizeof(int));
    }
    if (in_static && total > kStaticTableBytes) {
        delete bt;
        return fail(nullptr, STENCIL_EINVAL,
                    "the batch's descriptor table needs " + std::to_string(total) + " bytes; the static table holds " +
                        std::to_string(kStaticTableBytes) + " (fewer shots, or stencil_batch_create)");
    }
    std::unique_lock<std::mutex> lock(g_static_mu, std::defer_lock);
    if (!bt->groups.empty()) {
        DeviceGuard guard(bt->device);
        hipError_t he = guard.status;
        char *p = nullptr;
        if (he == hipSuccess && in_static) {
            lock.lock();
            void *base = nullptr;
            he = static_table(bt->device, &base);
            p = (char *)base;
        } else if (he == hipSuccess) {
            he = hipMalloc(&bt->dmem, total);
            p = (char *)bt->dmem;
        }
        if (he != hipSuccess) {
            delete bt;
            return hip_fail(nullptr, he, in_static ? "static batch table address" : "batch table allocation");
        }
        for (size_t gi = 0; gi < bt->groups.size(); ++gi) {
            auto &g = bt->groups[gi];
            for (int par = 0; par < 2; ++par) {
                g.tab[par] = (SweepArgs *)p;
                size_t sz = tabs[par][gi].size() * sizeof(SweepArgs);
                hipError_t he = hipMemcpy(p, tabs[par][gi].data(), sz, hipMemcpyHostToDevice);
                if (he != hipSuccess) {
                    if (bt->dmem) hipFree(bt->dmem);
                    delete bt;
                    return hip_fail(nullptr, he, "batch table upload");
                }
                p += round256(sz);
            }
            g.begin = (int *)p;
            size_t sz = begins[gi].size() * sizeof(int);
            hipError_t he = hipMemcpy(p, begins[gi].data(), sz, hipMemcpyHostToDevice);
            if (he != hipSuccess) {
                if (bt->dmem) hipFree(bt->dmem);
                delete bt;
                return hip_fail(nullptr, he, "batch table upload");
            }
            p += round256(sz);
        }
    }
    if (in_static) {
        // A batch without z-march groups does not touch the table, but it
        // still replaces the contents' owner, so that the rule "the latest
        // static batch on a device is the one that runs" has no exception.
        if (!lock.owns_lock()) lock.lock();
        if (bt->device < 0 || bt->device >= kMaxDevices) {
            delete bt;
            return fail(nullptr, STENCIL_EINVAL, "device number outside 0..63");
        }
        bt->in_static = true;
        bt->generation = ++g_static_gen[bt->device];
    }
    *out = bt;
    return STENCIL_OK;
}

}  // namespace

stencil_status stencil_batch_create(const stencil_shot *shots, int32_t n, int64_t it0, stencil_batch **out)
{
    return build_batch(shots, n, nullptr, it0, out);
}

stencil_status stencil_batch_create_static(const stencil_shot *shots, int32_t n, int64_t it0, stencil_batch **out)
{
    return build_batch(shots, n, nullptr, it0, out, true);
}

stencil_status stencil_batch_step(stencil_batch *bt, int64_t it, void *stream)
{
    if (!bt) return STENCIL_EINVAL;
    if (it < bt->it0 || it >= bt->nt_min) return STENCIL_EINVAL;
    if (bt->in_static) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_gen[bt->device] != bt->generation)
            return fail(nullptr, STENCIL_EINVAL,
                        "a later stencil_batch_create_static on this device replaced this batch's static table");
    }
    const int par = (int)((it - bt->it0) & 1);
    DeviceGuard guard(bt->device);
    if (guard.status != hipSuccess) return STENCIL_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    for (auto &g : bt->groups) {
        hipError_t e = p1310::launch_zmarch_batch(*g.v, g.tab[par], g.begin, g.nshots, g.blocks, g.xcd, it, s);
        if (e != hipSuccess) return STENCIL_EDEVICE;
    }
    for (size_t i = 0; i < bt->shots.size(); ++i) {
        const auto &sh = bt->shots[i];
        const void *uc = par ? sh.u_b : sh.u_a;
        void *up = par ? sh.u_a : sh.u_b;
        const bool solo = sh.tile.kind != STENCIL_TILE_ZMARCH;
        if (solo) {
            hipError_t e = enqueue_step(sh.ctx, sh.tile, sh.kappa, uc, up, up, it, sh.src.n ? &sh.src : nullptr, s);
            if (e != hipSuccess) return STENCIL_EDEVICE;
        } else if (sh.src.n > 1) {
            hipError_t e = p1310::launch_inject(sh.ctx->st, up, sh.kappa, nstore(sh.ctx), sh.ctx->pitch, sh.ctx->d.nx,
                                                sh.src.idx, sh.src.amp,
                                                sh.src.n, it, sh.ctx->scale, s);
            if (e != hipSuccess) return STENCIL_EDEVICE;
        }
    }
    return STENCIL_OK;
}

int32_t stencil_batch_launches(const stencil_batch *bt)
{
    if (!bt) return STENCIL_EINVAL;
    int32_t k = (int32_t)bt->groups.size() + (int32_t)bt->solo.size();
    for (const auto &sh : bt->shots)
        if (sh.tile.kind == STENCIL_TILE_ZMARCH && sh.src.n > 1) ++k;
    return k;
}

void stencil_batch_destroy(stencil_batch *bt)
{
    if (!bt) return;
    if (bt->dmem) {
        DeviceGuard guard(bt->device);
        (void)hipFree(bt->dmem);
    }
    delete bt;
}

stencil_status stencil_batch_tune(const stencil_shot *shots, int32_t n, const stencil_tune_opts *opts,
                                  stencil_tune_report *report, void *stream)
{
    if (!shots || n < 1 || n > 4096 || !report || !shots[0].ctx) return STENCIL_EINVAL;
    stencil_tune_opts o = {};
    if (opts) o = *opts;
    if (o.policy < STENCIL_POLICY_WORST || o.policy > STENCIL_POLICY_OB || o.n_iter < 0 || o.n_rep < 0 ||
        o.parts < 0 || o.parts == 1 || o.table_cap < 0)
        return fail(nullptr, STENCIL_EINVAL, "bad tune options");
    const int n_iter = o.n_iter ? o.n_iter : 10;
    const int n_rep = o.n_rep ? o.n_rep : 3;
    const int warm = o.warmup == 0 ? 2 : (o.warmup < 0 ? 0 : o.warmup);
    *report = stencil_tune_report{};
    const auto t_start = std::chrono::steady_clock::now();
    // Timing copies of the shots without sources.
    std::vector<stencil_shot> quiet(shots, shots + n);
    for (auto &q : quiet) q.src = stencil_src{};
    {
        // The shots as given must form a batch (no null or aliased fields).
        stencil_batch *probe = nullptr;
        const stencil_status st = build_batch(quiet.data(), n, nullptr, 0, &probe);
        if (st != STENCIL_OK) return fail(nullptr, st, "the shots do not form a batch (null, aliased or mixed devices)");
        stencil_batch_destroy(probe);
    }
    // Candidates: those of the first shot that every shot can run.
    std::vector<stencil_tile> base = make_candidates(shots[0].ctx, o);
    std::vector<std::vector<stencil_tile>> cands;  // per candidate: one tile per shot
    std::vector<stencil_tile> cand_key;
    for (const auto &t : base) {
        std::vector<stencil_tile> per(n);
        bool ok = true;
        for (int i = 0; i < n && ok; ++i) {
            std::string keep = shots[i].ctx->err;
            ok = check_tile(shots[i].ctx, t, &per[i]) == STENCIL_OK;
            shots[i].ctx->err = keep;
        }
        if (ok) {
            cands.push_back(per);
            cand_key.push_back(t);
        }
    }
    const int nC = (int)cands.size();
    if (nC == 0) return fail(nullptr, STENCIL_EUNSUPPORTED, "no tile fits every shot");
    DeviceGuard g(shots[0].ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(nullptr, g.status, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(nullptr, he, "hipEventCreate");
    he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(nullptr, he, "hipEventCreate");
    }
    auto time_batch = [&](const stencil_tile *tiles) -> double {
        stencil_batch *bt = nullptr;
        if (build_batch(quiet.data(), n, tiles, 0, &bt) != STENCIL_OK) return std::numeric_limits<double>::infinity();
        double ms = std::numeric_limits<double>::infinity();
        bool okk = true;
        for (int i = 0; i < warm && okk; ++i) okk = stencil_batch_step(bt, i, s) == STENCIL_OK;
        if (okk) {
            hipEventRecord(e0, s);
            for (int i = 0; i < n_iter && okk; ++i) okk = stencil_batch_step(bt, warm + i, s) == STENCIL_OK;
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) == hipSuccess && okk) {
                float f = 0;
                hipEventElapsedTime(&f, e0, e1);
                ms = f;
            }
        }
        stencil_batch_destroy(bt);
        return ms;
    };
    std::vector<double> table((size_t)n_rep * nC, std::numeric_limits<double>::infinity());
    for (int r = 0; r < n_rep; ++r)
        for (int c = 0; c < nC; ++c) table[(size_t)r * nC + c] = time_batch(cands[c].data());
    bool any = false;
    for (double v : table) any = any || std::isfinite(v);
    if (!any) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return fail(nullptr, STENCIL_EDEVICE, "every batch candidate failed");
    }
    int32_t best = 0;
    double min_time = 0;
    stencil_select(table.data(), 1, n_rep, nC, o.policy, &best, &min_time);
    const double actual = time_batch(cands[best].data());
    const double dtime = time_batch(nullptr);  // the shots' own tiles
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (int i = 0; i < n; ++i) shots[i].ctx->tile = cands[best][i];
    if (log_on())
        std::fprintf(stderr, "stencil: batch tune, %d shots: %d candidates x %d replicates x %d steps, chose %s, "
                     "MinTime %.4f ms, ActualTime %.4f ms\n", n, nC, n_rep, n_iter, tile_text(cand_key[best]).c_str(),
                     min_time, actual);
    report->tile = cand_key[best];
    report->min_time_ms = min_time;
    report->actual_time_ms = actual;
    report->gap = (actual - min_time) / min_time;
    report->default_time_ms = dtime;
    report->n_candidates = nC;
    report->from_cache = 0;
    report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (o.table && o.table_cap > 0)
        for (int r = 0; r < n_rep; ++r)
            for (int c = 0; c < nC && c < o.table_cap; ++c) o.table[(size_t)r * o.table_cap + c] = table[(size_t)r * nC + c];
    if (o.candidates)
        for (int c = 0; c < nC && c < o.table_cap; ++c) o.candidates[c] = cand_key[c];
    return STENCIL_OK;
}

stencil_status stencil_convert(stencil_ctx *ctx, const void *src, void *dst, int32_t to_storage, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!src || !dst) return fail(ctx, STENCIL_EINVAL, "null pointer");
    const int64_t ub = nstore(ctx) * ctx->es, fb = nstore(ctx) * 4;
    if (overlaps2(src, to_storage ? fb : ub, dst, to_storage ? ub : fb))
        return fail(ctx, STENCIL_EALIAS, "src and dst overlap");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = p1310::launch_convert(ctx->st, src, dst, nstore(ctx), ctx->scale, to_storage ? 1 : 0,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "convert launch");
    return STENCIL_OK;
}

stencil_status stencil_stream_probe(const void *a, const void *b, const void *c, void *out, int64_t nbytes,
                                    void *stream)
{
    if (!a || !out || (c && !b) || nbytes <= 0 || nbytes % 4 ||
        (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)out) & 3u))
        return STENCIL_EINVAL;
    hipError_t e = p1310::launch_stream(a, b, c, out, nbytes, (hipStream_t)stream);
    return e == hipSuccess ? STENCIL_OK : STENCIL_EDEVICE;
}

stencil_status stencil_max_abs(stencil_ctx *ctx, const void *u, float *out, void *stream)
{
    if (!ctx) return STENCIL_EINVAL;
    if (!u || !out) return fail(ctx, STENCIL_EINVAL, "null pointer");
    if (overlaps2(out, 4, u, nstore(ctx) * ctx->es)) return fail(ctx, STENCIL_EALIAS, "out lies inside the field");
    DeviceGuard g(ctx->d.device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipError_t e = p1310::launch_max_abs(ctx->st, u, nstore(ctx), (unsigned int *)out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "max_abs launch");
    return STENCIL_OK;
}

stencil_status stencil_stream_probe_march(const void *a, const void *b, const void *c, void *out, int64_t nx,
                                          int64_t ny, int64_t nz, void *stream)
{
    if (!a || !b || !c || !out || nx < 4 || nx % 4 || ny < 1 || nz < 1 || nx > 0x7fffffff || ny > 0x7fffffff ||
        nz > 0x7fffffff || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)out) & 15u))
        return STENCIL_EINVAL;
    const int64_t bytes = nx * ny * nz * 4;
    if (overlaps(a, out, bytes) || overlaps(b, out, bytes) || overlaps(c, out, bytes)) return STENCIL_EALIAS;
    hipError_t e = p1310::launch_stream_march(a, b, c, out, nx, ny, nz, (hipStream_t)stream);
    return e == hipSuccess ? STENCIL_OK : STENCIL_EDEVICE;
}

}  // extern "C"
