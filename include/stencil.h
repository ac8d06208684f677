/*
 * C ABI of the MI355X (gfx950) blocked star-stencil library
 * (libpaper_1310_8232_amd.so).
 *
 * The operation (paper: Section 2, the "3D model" step inside the time loop
 * of Algorithm 1; 10th order in space, 2nd order in time; star stencil with
 * neighbours along both directions of all three axes, Fig. 1(a)):
 *
 *   L u(p)   = sum_{d in x,y,z} [ c_0 u(p) + sum_{m=1..R} c_m (u(p + m e_d) + u(p - m e_d)) ]
 *   u^{n+1}  = 2 u^n - u^{n-1} + kappa * L u^n,     kappa = (v dt / h)^2
 *   u^{n+1}(s_j) += kappa(s_j) * amp[n][j]           (point sources)
 *
 * u is 0 outside the grid (zero Dirichlet ghost layer); every grid point is
 * updated. c_m are the order-2R central second-difference weights. The
 * paper's loop blocking (Section 3, Fig. 1(b)) becomes the workgroup tile;
 * its blocksize search (Sections 3.2-3.3, 3.6, 3.7) becomes stencil_tune.
 *
 * Data layout: every field is a contiguous array [nz][ny][pitch] in device
 * memory, x unit-stride, point (z, y, x) at linear index
 * (z*ny + y)*pitch + x, where pitch = nx unless stencil_desc.pitch sets a
 * longer row (caller-padded rows, e.g. to a multiple of 128 bytes so that
 * every row starts on a cache line). Values x in [nx, pitch) of a row are
 * padding: the sweeps neither read them as grid points nor write them; the
 * element-wise calls (kappa, convert, gradient terms, max |u|) process them
 * like any other value, so keep them finite (zero). Source and receiver
 * indices are linear indices of this layout; one that falls in padding is
 * skipped (sources) or samples 0 (receivers). kappa and the gradient fields
 * are FP32 / FP64, wavefields are in the context's storage type (FP32 unless
 * FP16/BF16 is chosen). Sizes below ("of the grid's shape") mean
 * pitch*ny*nz values.
 *
 * Ownership: field pointers are borrowed device memory (e.g. torch tensors);
 * the library never allocates, frees or retains them. A context owns only
 * host state (sizes, coefficients, the chosen tile). Contexts are not
 * thread-safe; separate contexts are independent.
 *
 * Errors: every call returns a stencil_status (0 = success, negative =
 * failure). Arguments are validated before any launch; a failed call leaves
 * the fields untouched and records a message readable with
 * stencil_last_error. No C++ exception crosses this interface.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream). The stepping calls (stencil_kappa, stencil_step, stencil_step_to,
 * stencil_step2, stencil_adjoint_step, stencil_gradient2, stencil_gradient_terms,
 * stencil_sample, stencil_misfit, stencil_convert, stencil_batch_step,
 * stencil_max_abs) only enqueue work: no
 * allocation, no synchronisation, no host read of device memory, so they may
 * be captured in a HIP graph. stencil_tune and stencil_batch_tune synchronise
 * the stream.
 */
#ifndef PAPER_1310_8232_AMD_STENCIL_H
#define PAPER_1310_8232_AMD_STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STENCIL_OK = 0,
    STENCIL_EINVAL = -1,        /* bad argument: size, radius, pointer, alignment, step index */
    STENCIL_EUNSTABLE = -2,     /* vmax*dt/h above the leapfrog stability limit */
    STENCIL_ENOMEM = -3,        /* host allocation failed */
    STENCIL_EDEVICE = -4,       /* a HIP call failed (message in stencil_last_error) */
    STENCIL_EUNSUPPORTED = -5,  /* storage type or tile the library has no compiled kernel for */
    STENCIL_EALIAS = -6,        /* fields that must be distinct overlap (e.g. u_cur and the output) */
    STENCIL_EDIVERGED = -7      /* a wavefield is no longer finite or exceeds a caller's limit (not
                                   returned by the library's calls: see stencil_max_abs) */
} stencil_status;

typedef struct stencil_ctx stencil_ctx;  /* opaque */
typedef struct stencil_batch stencil_batch;  /* opaque */

/* Wavefield storage (kappa is always FP32; arithmetic is always FP32). The
 * 16-bit types hold storage_scale * u, widened to FP32 on load and rounded to
 * nearest even once per store; available for R = 4 and 5. */
typedef enum { STENCIL_F32 = 0, STENCIL_F16 = 1, STENCIL_BF16 = 2 } stencil_storage;

typedef enum {
    STENCIL_TILE_AUTO = 0,   /* the context's current tile (tuned, cached or built-in default) */
    STENCIL_TILE_PLAIN = 1,  /* plain tiling: one thread per point, workgroup bx*by*dz, taps read from memory */
    STENCIL_TILE_ZMARCH = 2, /* xy tile staged in LDS, register queue marching dz planes along z */
    STENCIL_TILE_ZMARCH2 = 3 /* two leapfrog steps per launch (blocking in time): see stencil_step2 */
} stencil_tile_kind;

/* The GPU form of the paper's blocksize (bi, bj, bk). For ZMARCH a workgroup
 * of bx*by threads owns a (bx*vw) x (by*ry) tile in (x, y) and marches dz
 * planes in z; each thread computes vw consecutive x points of ry
 * consecutive rows. For PLAIN a workgroup is bx x by x dz threads. */
typedef struct {
    int32_t kind;   /* stencil_tile_kind */
    int32_t bx;     /* threads along x */
    int32_t by;     /* threads along y */
    int32_t ry;     /* rows per thread along y (ZMARCH) */
    int32_t dz;     /* planes per workgroup along z (ZMARCH); threads along z (PLAIN) */
    int32_t vw;     /* x points per thread: 8 (ZMARCH, 16-bit storage), 4, 2 (ZMARCH, FP32
                       storage) or 1; must divide nx and the pitch; 0 = the widest that does */
    int32_t xcd;    /* 1 = XCD-aware workgroup order (neighbour tiles share an L2) */
    int32_t pf;     /* bit 0: 1 = prefetch u^{n-1} and kappa one plane ahead (ZMARCH, ZMARCH2).
                       ZMARCH2 only, bits 1-3: edge pacing code p in 0..7: with at least
                       three tile columns, the workgroups of the first and last column
                       pause about 4p x 64 cycles per plane (0 = off), so that they keep
                       step with their neighbours (see stencil_step2) */
} stencil_tile;

typedef struct {
    int64_t nx, ny, nz;   /* grid points, each >= 1 */
    int32_t radius;       /* R in {3, 4, 5}: order 2R in space (4 = 8th order, 25 points; 5 = the paper's 10th) */
    int32_t storage;      /* stencil_storage */
    double h;             /* grid spacing (isotropic), > 0 */
    double dt;            /* time step, > 0 */
    double vmax;          /* largest velocity of the model, > 0, used for the stability check */
    int32_t device;       /* HIP device ordinal of the fields */
    stencil_tile tile;    /* kind 0 = tune cache entry if any, else the built-in default */
    double storage_scale; /* wavefields are stored as storage_scale * u; a power of two (0 = 1).
                             The scheme is linear, so only source amplitudes are multiplied by it. */
    int64_t pitch;        /* row stride in values: 0 = nx, else >= nx (padded rows). Vector tiles
                             need vw to divide the pitch as well as nx. */
} stencil_desc;

/* Point sources (all device memory, borrowed): idx[n] linear indices,
 * amp[nt][n] samples; step `it` adds kappa(idx[j]) * amp[it*n + j] to
 * u^{it+1}(idx[j]) for j = 0..n-1 in order (an index may repeat; its terms
 * are added in that order). Indices outside the grid are skipped by the
 * kernels. One source is added inside the sweep; n > 1 costs one more launch
 * per step in which every workgroup of 256 sources reads all n indices once. */
typedef struct {
    int32_t n;
    const int64_t *idx;
    const float *amp;
    int64_t nt;
} stencil_src;

typedef enum {
    STENCIL_POLICY_WORST = 0,  /* MWMB (Eq. 2): worst of the per-replicate minima; the default */
    STENCIL_POLICY_MIN = 1,    /* MMMB (Eq. 1) */
    STENCIL_POLICY_AVG = 2,    /* MAMB (Eq. 3) */
    STENCIL_POLICY_OB = 3      /* Original Block: fastest single measurement */
} stencil_policy;

typedef struct {
    int32_t policy;          /* stencil_policy */
    int32_t n_iter;          /* nI: timed steps per candidate (Section 3.2); 0 = 10 */
    int32_t n_rep;           /* replicate passes over the same candidate list in the same order; 0 = 3 */
    int32_t warmup;          /* untimed steps before each timing; 0 = 2, -1 = none */
    int32_t parts;           /* 0 = every legal tile x the dz list; P >= 2 = Section 3.7's P-part grid */
    int32_t include_plain;   /* 1 = also time plain-tiling candidates */
    const char *cache_path;  /* tune cache file (read before, written after); NULL = none. Only
                                entries written by a library with the same stencil_build_id are read */
    double *table;           /* optional out: [n_rep][table_cap] times in ms (row-major) */
    stencil_tile *candidates;/* optional out: [table_cap] candidate tiles in timing order */
    int32_t table_cap;
    int32_t temporal;        /* 0/1 = one-step tiles (the context's tile); 2 = two-step tiles (its tile2,
                                times still per n_iter steps, n_iter rounded up to even) */
    void *scratch_c;         /* two-step search: two more scratch fields of the grid's shape */
    void *scratch_d;
} stencil_tune_opts;

typedef struct {
    stencil_tile tile;       /* chosen tile (also made the context's current tile) */
    double min_time_ms;      /* MinTime: selection-phase time of n_iter steps */
    double actual_time_ms;   /* ActualTime: verification-phase time of n_iter steps */
    double gap;              /* (ActualTime - MinTime) / MinTime (Section 3.6) */
    double default_time_ms;  /* n_iter steps with the built-in default tile, same conditions */
    double seconds;          /* wall time of the whole search */
    int32_t n_candidates;    /* nC */
    int32_t from_cache;      /* 1 = taken from cache_path without timing */
} stencil_tune_report;

/* Create a context. Validates sizes, radius, storage, h, dt, vmax (> 0) and
 * the stability limit vmax*dt/h <= stencil_cfl_limit(radius) (EUNSTABLE).
 * Host-only: no device call. *out is set only on success.
 * Environment: STENCIL_TUNE_CACHE names a tune cache file whose last entry
 * for this grid, radius and storage, written by a library with the same
 * stencil_build_id, gives the initial tile when d->tile is kind 0 (unreadable
 * lines, entries of another build and tiles no kernel runs are ignored:
 * built-in default); STENCIL_LOG (anything but empty or "0") prints one line to stderr
 * per context created and per search (stencil_tune, stencil_batch_tune). */
stencil_status stencil_init(const stencil_desc *d, stencil_ctx **out);

/* Release a context (NULL is ignored). */
void stencil_destroy(stencil_ctx *ctx);

/* kappa(p) = (v(p) dt / h)^2 for every point, formed in FP64 and rounded
 * once to FP32 (the model set-up of Section 2's scheme). v and kappa are
 * device arrays of the grid's shape; they may be the same array. */
stencil_status stencil_kappa(stencil_ctx *ctx, const void *v, void *kappa, void *stream);

/* (Wavefield arguments of the stepping calls are in the context's storage
 * type; with a tile of vw > 1 they must be aligned to vw values and kappa
 * to 4*vw bytes, else EINVAL.) */

/* stencil_step with the output in its own buffer: reads u_cur = u^{it} and
 * u_prev = u^{it-1}, writes u^{it+1} (sources included) to u_next. u_next may
 * be u_prev (the in-place form) but must not otherwise overlap u_prev, and
 * must not overlap u_cur or kappa (EALIAS). Same traffic as the in-place form. */
stencil_status stencil_step_to(stencil_ctx *ctx, const void *kappa, const void *u_cur, const void *u_prev,
                               void *u_next, int64_t it, const stencil_src *src, void *stream);

/* Two leapfrog steps in one launch (blocking in time as well as in space):
 * reads u_cur = u^{it}, u_prev = u^{it-1}, kappa; writes u^{it+1} to u_next
 * and u^{it+2} to u_next2, with the sources of steps it and it+1. The four
 * wavefields must be distinct and must not overlap (EALIAS): the inputs are
 * read around every tile by its neighbours while the outputs are written.
 * At most one source (EUNSUPPORTED otherwise; a negative count is EINVAL);
 * it+1 < src->nt (EINVAL).
 * Results are bit-identical to two stencil_step calls. Uses the context's
 * two-step tile; FP32 storage. Capture-safe. Edge pacing (tile.pf bits 1-3):
 * the tiles of the grid's first and last tile column have out-of-grid halo
 * columns, which cost no memory traffic, so they march ahead of their
 * neighbours, and the halo lines the two share are then fetched twice
 * instead of being found in the L2; a short pause per plane in those tiles
 * keeps them in step. It changes timing only, never results; the search
 * (stencil_tune with temporal = 2) times paced and unpaced tiles. */
stencil_status stencil_step2(stencil_ctx *ctx, const void *kappa, const void *u_cur, const void *u_prev,
                             void *u_next, void *u_next2, int64_t it, const stencil_src *src, void *stream);

/* One leapfrog step n = it: reads u_cur = u^{it} and u_prev_next = u^{it-1},
 * overwrites u_prev_next with u^{it+1}, then injects the sources (src may
 * be NULL). Requires it < src->nt when src is given (EINVAL). u_cur and
 * u_prev_next must not overlap (EALIAS); kappa must not overlap
 * u_prev_next. Pointers must be aligned to vw values (kappa: 4*vw bytes)
 * when the tile uses vw > 1. */
stencil_status stencil_step(stencil_ctx *ctx, const void *kappa, const void *u_cur,
                            void *u_prev_next, int64_t it, const stencil_src *src, void *stream);

/* kappa(p) = dt^2 / (h^2 m(p)) from squared slowness m = 1/v^2 (the model
 * parameter of the gradient below), formed in FP64 and rounded once. */
stencil_status stencil_kappa_slowness2(stencil_ctx *ctx, const void *m, void *kappa, void *stream);

/* Receiver samples out[j] = u[idx[j]] for j < n (FP32; 0 for an index outside
 * the grid). idx and out are device arrays of n entries. FP32 storage only
 * (EUNSUPPORTED otherwise); so is stencil_adjoint_step. */
stencil_status stencil_sample(stencil_ctx *ctx, const void *u, const int64_t *idx, int32_t n, void *out,
                              void *stream);

/* One step of the discrete adjoint of stencil_step, run backward in time.
 * For the misfit J = 1/2 sum_k sum_r (u^k(r) - d^k(r))^2 the Lagrange
 * multipliers obey lambda^k = 2 lambda^{k+1} - lambda^{k+2} + L(kappa lambda^{k+1}) + r^k
 * (L symmetric); the library carries mu = kappa * lambda, whose recurrence
 * mu^k = 2 mu^{k+1} - mu^{k+2} + kappa L mu^{k+1} + kappa r^k is the forward
 * step with the residuals injected at the receivers. So: lam_cur = mu^{k+1},
 * lam_prev_next = mu^{k+2} on entry and mu^k on exit, resid = receivers with
 * residual rows (row `it` is injected; it = k-1 for traces recorded as row
 * k-1 = u^k), same rules as stencil_step.
 * If grad != NULL (FP64, [nz][ny][nx]) it also accumulates the gradient with
 * respect to squared slowness m = 1/v^2:
 *   grad += -(h^2/dt^2) * mu^k * (u_next - 2 u_cur + u_prev)
 * with u_next = u^k, u_cur = u^{k-1}, u_prev = u^{k-2} (FP32 fields); summed
 * over k = N..1 this is dJ/dm. grad must not overlap any other field
 * (EALIAS). */
stencil_status stencil_adjoint_step(stencil_ctx *ctx, const void *kappa, const void *lam_cur, void *lam_prev_next,
                                    int64_t it, const stencil_src *resid, const void *u_next, const void *u_cur,
                                    const void *u_prev, double *grad, void *stream);

/* The gradient terms of two consecutive adjoint steps k and k-1 (each run
 * with grad = NULL) in one pass over memory:
 *   grad += -(h^2/dt^2) * mu^k     * (u^k     - 2 u^{k-1} + u^{k-2})
 *   grad += -(h^2/dt^2) * mu^{k-1} * (u^{k-1} - 2 u^{k-2} + u^{k-3})
 * in this order, each term rounded as stencil_adjoint_step rounds it, so the
 * result is the bits of the two accumulating adjoint steps. After the two
 * steps mu^k is in their lam_cur buffer and mu^{k-1} in lam_prev_next. FP32
 * fields, FP64 grad (must not overlap another field: EALIAS); FP32 storage
 * only (EUNSUPPORTED). Capture-safe. */
stencil_status stencil_gradient2(stencil_ctx *ctx, const void *mu_k, const void *mu_km1, const void *u_k,
                                 const void *u_km1, const void *u_km2, const void *u_km3, double *grad, void *stream);

/* m = 1..4 consecutive gradient terms in one pass, for adjoint steps k,
 * k-1, ..., k-m+1: grad += s mu[j] ((u[j] - 2 u[j+1]) + u[j+2]) for
 * j = 0, 1, ..., m-1 in that order, s = -h^2/dt^2, each term formed in FP64
 * and added as stencil_adjoint_step adds it, so the result has the bits of m
 * single-term accumulations (stencil_gradient2 is m = 2). mu is a host array
 * of m device pointers (mu^k, mu^{k-1}, ...), u a host array of m + 2
 * (u^k, u^{k-1}, ..., u^{k-m-1}); FP32 fields of the grid, FP64 grad, which
 * must not overlap another field (EALIAS). FP32 storage; capture-safe. Per
 * point (2m + 2) x 4 B read and 16 B of grad read and written. */
stencil_status stencil_gradient_terms(stencil_ctx *ctx, int32_t m, const void *const *mu, const void *const *u,
                                      double *grad, void *stream);

/* resid[i] = traces[i] - observed[i] (FP32, i < count; resid may be NULL) and
 * *misfit = 1/2 sum resid^2 accumulated in FP64 in a fixed order (device
 * double). All pointers are device memory; with count = 0 traces and
 * observed may be NULL and *misfit is set to 0. */
stencil_status stencil_misfit(const void *traces, const void *observed, int64_t count, void *resid, double *misfit,
                              void *stream);

/* One shot of a batch: its context (grid, weights, current tile), kappa and
 * two wavefield buffers (device, borrowed), and its sources (src.n = 0 for
 * none; idx/amp device pointers as in stencil_src). */
typedef struct {
    stencil_ctx *ctx;
    const void *kappa;
    void *u_a;
    void *u_b;
    stencil_src src;
} stencil_shot;

/* Several independent grids (shots, each with its own size and tuned tile)
 * advanced together. Shots whose tiles use the same compiled kernel are swept
 * by one launch per step (the launch grid concatenates their workgroups; each
 * keeps its own march depth); plain-tile shots get a launch of their own.
 * Copies each context's current tile; allocates one small device table
 * (hipMalloc, here only). Buffers alternate: at step `it` with
 * (it - it0) even, u_a holds u^{it}, u_b holds u^{it-1} and receives u^{it+1};
 * with (it - it0) odd the roles swap. Rejects (EINVAL / EALIAS) a null shot,
 * a shot whose buffers overlap each other or its kappa, a buffer that overlaps
 * any field of another shot (shots may share one kappa, which is only read),
 * and mixed devices. */
stencil_status stencil_batch_create(const stencil_shot *shots, int32_t n, int64_t it0, stencil_batch **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batch as stencil_batch_create, whose descriptor table (the only device
 * memory a batch uses beyond the shots' own fields) is placed in a
 * library-owned static device array of 64 KiB per GPU instead of a
 * hipMalloc'd one. Calls no hipMalloc/hipFree (host bookkeeping only);
 * uploads the table with hipMemcpy. Limits: the table takes 2 x 144 B per
 * z-march shot plus 4 B, each of a kernel group's three parts rounded up to
 * 256 B, so 224 shots of one tile shape fit; a larger batch is refused with EINVAL and a message
 * (stencil_last_error(NULL)) before any device call. Every static batch on a
 * GPU shares that GPU's array: creating one replaces the table of the
 * previous one, whose later stencil_batch_step calls return EINVAL. The
 * caller must not create a static batch while steps of an earlier static
 * batch on that GPU may still run (such calls overlap and race). Steps,
 * launches count and destroy are as for stencil_batch_create. */
stencil_status stencil_batch_create_static(const stencil_shot *shots, int32_t n, int64_t it0, stencil_batch **out);

/* One step of every shot of the batch on `stream`; capture-safe (no
 * allocation, no synchronisation). EINVAL if it < it0 or it reaches the
 * shortest source length, or for a static batch whose table a later
 * stencil_batch_create_static on the same GPU replaced. */
stencil_status stencil_batch_step(stencil_batch *b, int64_t it, void *stream);

/* The blocksize search of stencil_tune run on a whole batch: every candidate
 * tile (those of the first shot's search that every shot can run) is applied
 * to all shots at once and timed as a batch step, so the choice is made under
 * the contention of the production run (the situation that motivates the
 * same-order evaluation of Section 3.3). The shots' u_a/u_b are used as
 * scratch and overwritten; sources are not injected while timing. Sets every
 * shot's context tile to the winner and fills *report
 * (default_time_ms = the shots' own tiles). opts may be NULL; cache_path is
 * ignored. Synchronises `stream`. */
stencil_status stencil_batch_tune(const stencil_shot *shots, int32_t n, const stencil_tune_opts *opts,
                                  stencil_tune_report *report, void *stream);

/* Kernel launches one batch step issues. */
int32_t stencil_batch_launches(const stencil_batch *b);

/* Release a batch (NULL is ignored). Does not free the shots' buffers. */
void stencil_batch_destroy(stencil_batch *b);

/* The paper's two-phase blocksize search (Sections 3.2-3.3) on the
 * production shape: the selection phase times every candidate for n_iter
 * steps, n_rep times in the same fixed order, and reduces the table with
 * opts->policy; the verification phase re-times the winner (ActualTime).
 * scratch_a/scratch_b are device fields of the grid's shape used as u^n and
 * u^{n-1}: their contents are overwritten. Synchronises `stream`. Sets the
 * context's tile and fills *report. opts may be NULL (defaults). */
stencil_status stencil_tune(stencil_ctx *ctx, const void *kappa, void *scratch_a, void *scratch_b,
                            const stencil_tune_opts *opts, stencil_tune_report *report, void *stream);

/* Current one-step tile of the context (after init, tune or set). */
stencil_status stencil_get_tile(const stencil_ctx *ctx, stencil_tile *out);

/* Current two-step tile (EUNSUPPORTED if no two-step kernel exists for the
 * context's radius and storage). */
stencil_status stencil_get_tile2(const stencil_ctx *ctx, stencil_tile *out);

/* Replace the current tile (a ZMARCH2 tile replaces the two-step tile);
 * rejects tiles the compiled kernels cannot run on the context's grid
 * (EUNSUPPORTED) without changing the current one: no compiled kernel for the
 * shape, vw not dividing nx, a z window of 2 GiB or more, or a launch of more
 * than 2^31-1 workgroups or 2^32-1 work-items. */
stencil_status stencil_set_tile(stencil_ctx *ctx, const stencil_tile *tile);

/* Compiled ZMARCH tiles for a radius and storage type, with vw = 4
 * (vec4 = 1), 8 (vec4 = 8), 2 (vec4 = 2) or 1 (vec4 = 0), dz = 0. Writes at
 * most cap entries to out (out may be NULL) and returns the total count, or a
 * negative stencil_status. */
int32_t stencil_list_tiles(int32_t radius, int32_t vec4, int32_t storage, stencil_tile *out, int32_t cap);

/* Compiled two-step tiles (kind ZMARCH2, dz = 0) for a radius, FP32 storage. */
int32_t stencil_list_tiles2(int32_t radius, int32_t vec4, stencil_tile *out, int32_t cap);

/* Between FP32 wavefields and the context's storage: to_storage != 0 writes
 * dst = round(src * storage_scale) (nearest even) in the storage type;
 * to_storage = 0 writes FP32 dst = src / storage_scale. Whole grid, device
 * memory, no overlap (EALIAS). */
stencil_status stencil_convert(stencil_ctx *ctx, const void *src, void *dst, int32_t to_storage, void *stream);

/* FP32 weights the kernels use: out[0] = 3*c_0, out[m] = c_m (m = 1..R).
 * Returns R+1, or EINVAL for an unsupported radius. */
int32_t stencil_coefficients(int32_t radius, float *out);

/* Largest stable v*dt/h for the radius (2 / sqrt(3 |c_0 + 2 sum_m (-1)^m c_m|)),
 * or a negative value for an unsupported radius. */
double stencil_cfl_limit(int32_t radius);

/* Section 3.3's three-stage reduction of a timing table, host only.
 * t[(i*n_cores + k)*n_cand + j] = time of candidate j of node i on core k;
 * node i's candidate j has global id i*n_cand + j. Stage 1: per-core
 * argmin; stage 2: per-node min / worst / closest-to-mean of the core
 * winners (policy); stage 3: argmin over nodes. STENCIL_POLICY_OB takes the
 * single smallest entry. Ties go to the lowest node, core, candidate.
 * Writes the chosen id and its time. */
stencil_status stencil_select(const double *t, int32_t n_nodes, int32_t n_cores, int32_t n_cand,
                              int32_t policy, int32_t *best_id, double *best_time);

/* Section 3.7's candidate list for one dimension of size S cut in P parts:
 * 1 + floor(j*S/(P-1)), j = 0..P-1, last clamped to S, repeats dropped.
 * Writes at most cap values and returns the count (or EINVAL). */
int32_t stencil_pgrid(int64_t S, int32_t P, int64_t *out, int32_t cap);

/* Streaming reference: out[i] = a[i] (+ b[i]) (+ c[i]) over nbytes of FP32
 * (a multiple of 4; 4-byte aligned device pointers; 16-byte vectors when the
 * size and every pointer allow; b may be NULL, c may be NULL, c non-NULL
 * needs b). With b = c = NULL it is a plain copy (used for wavefield
 * checkpoints); with all three it has the sweep's traffic mix of three reads
 * per write (the bandwidth reference). Enqueued on `stream`. */
stencil_status stencil_stream_probe(const void *a, const void *b, const void *c, void *out, int64_t nbytes,
                                    void *stream);

/* Divergence watchdog: the largest magnitude of the wavefield u (the
 * context's grid and storage type) into *out, a device float, in storage
 * units (storage_scale * |u| for 16-bit storage): NaN if any value is NaN,
 * +inf if any is infinite, else max |u|. Two launches on `stream` (a
 * one-thread clear of *out, then a grid-stride reduction with an atomic
 * maximum over the magnitude's bit pattern, which orders NaN above +inf above
 * every finite value); no allocation and no host wait, so it can be
 * captured. A caller checks *out every few steps and stops with
 * STENCIL_EDIVERGED when it is not finite or exceeds its limit. */
stencil_status stencil_max_abs(stencil_ctx *ctx, const void *u, float *out, void *stream);

/* Streaming reference in the one-step sweep's access order, without the
 * stencil: out = (a + b) + c over [nz][ny][nx] FP32 fields (nx % 4 == 0,
 * 16-byte aligned, out not overlapping an input: EINVAL / EALIAS), one
 * workgroup per column of 256 x 4 points marching 256 planes, a cached and
 * b, c, out non-temporal as in the sweep. The bandwidth ceiling of the
 * sweep's own access pattern. Enqueued on `stream`. */
stencil_status stencil_stream_probe_march(const void *a, const void *b, const void *c, void *out, int64_t nx,
                                          int64_t ny, int64_t nz, void *stream);

/* Identity of this library's code as the tune cache records it (static
 * storage): "<offload arch>/hip<compile-time HIP version>/rt<HIP runtime
 * version>/src<hash of the kernel and runtime sources>". A tile measured
 * with one build is not taken as the best tile of another. */
const char *stencil_build_id(void);

/* Message for a status code (static storage). */
const char *stencil_strerror(stencil_status s);

/* Last error message recorded on the context ("" if none); with ctx = NULL,
 * the calling thread's last message from calls that take no context
 * (batches, misfit, streaming reference). */
const char *stencil_last_error(const stencil_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1310_8232_AMD_STENCIL_H */
