/*
 * Plain FP64 CPU oracle for the leapfrog star-stencil wave step.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check and the CPU
 * baseline of the benchmark may load this file's library. The product path
 * (paper_1310_8232_amd/) never links, imports or calls it, and shares no
 * code, header, table or helper with it.
 *
 * What is computed (paper: Section 2, the "3D model" step of Algorithm 1,
 * a finite-difference scheme of high order in space and second order in
 * time, evaluated as a star stencil that weights neighbours along both
 * directions of all three axes, Fig. 1(a)):
 *
 *   Lu(p)    = sum over axes d of [ c0 u(p) + sum_{m=1..R} c_m (u(p+m e_d) + u(p-m e_d)) ]
 *   u^{n+1}  = 2 u^n - u^{n-1} + kappa * L u^n
 *   u^{n+1}(s) += kappa(s) * w_n               (point sources, after the update)
 *
 * with u taken as 0 outside the grid (zero Dirichlet ghost layer), grid index
 * p = (z*ny + y)*nx + x (x unit stride), kappa = (v dt / h)^2, and c_m the
 * standard central-difference weights of order 2R.
 *
 * Every loop is the plain definition: no blocking, no fusion, no reordering.
 * The only parallelism is an OpenMP split of the outer z loop over
 * independent points.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Coefficients. The paper uses order 10 in space (Section 2) and prints no  */
/* weights. Closed form of the order-2R central second-difference weights:   */
/*   c_m = 2 (-1)^{m+1} (R!)^2 / ( m^2 (R-m)! (R+m)! ),  m = 1..R           */
/*   c_0 = -2 sum_{m>=1} c_m                                                 */
/* Returns 0 on success, -1 for R outside 1..8.                              */
/* ------------------------------------------------------------------------- */
static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

int oracle_fd_coefficients(int R, double *c)
{
    if (R < 1 || R > 8) return -1;
    double rf = fact(R);
    double sum = 0.0;
    for (int m = 1; m <= R; ++m) {
        double sign = (m % 2 == 1) ? 1.0 : -1.0;
        c[m] = 2.0 * sign * rf * rf / ((double)m * (double)m * fact(R - m) * fact(R + m));
        sum += c[m];
    }
    c[0] = -2.0 * sum;
    return 0;
}

/* Stability limit of v*dt/h for the 3D leapfrog scheme: the largest |symbol|
 * of the 1D operator is at theta = pi, chat(pi) = c0 + 2 sum_m c_m (-1)^m;
 * the 3D operator's extreme eigenvalue is 3 chat(pi), and leapfrog is stable
 * while kappa * 3 |chat(pi)| <= 4, i.e. v dt / h <= 2 / sqrt(3 |chat(pi)|). */
double oracle_cfl_limit(int R)
{
    double c[9];
    if (oracle_fd_coefficients(R, c) != 0) return -1.0;
    double s = c[0];
    for (int m = 1; m <= R; ++m) s += 2.0 * c[m] * ((m % 2 == 0) ? 1.0 : -1.0);
    return 2.0 / sqrt(3.0 * fabs(s));
}

/* kappa(p) = (v(p) dt / h)^2 in FP64 from the FP32 velocity model. */
void oracle_kappa(int64_t n, const float *v, double dt, double h, double *kappa)
{
    for (int64_t i = 0; i < n; ++i) {
        double r = (double)v[i] * dt / h;
        kappa[i] = r * r;
    }
}

/* u(z, y, x) with the zero ghost layer outside the grid. */
static inline double at(const double *u, int64_t nx, int64_t ny, int64_t nz,
                        int64_t z, int64_t y, int64_t x)
{
    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return 0.0;
    return u[(z * ny + y) * nx + x];
}

/* Lu at one point, written exactly as the definition: a sum over the three
 * axes of the 1D stencil along that axis. */
static double lap_at(int R, const double *c, const double *u,
                     int64_t nx, int64_t ny, int64_t nz,
                     int64_t z, int64_t y, int64_t x)
{
    const int64_t dz[3] = {0, 0, 1}, dy[3] = {0, 1, 0}, dx[3] = {1, 0, 0};
    double total = 0.0;
    for (int d = 0; d < 3; ++d) {
        double axis = c[0] * at(u, nx, ny, nz, z, y, x);
        for (int m = 1; m <= R; ++m) {
            axis += c[m] * (at(u, nx, ny, nz, z + m * dz[d], y + m * dy[d], x + m * dx[d]) +
                            at(u, nx, ny, nz, z - m * dz[d], y - m * dy[d], x - m * dx[d]));
        }
        total += axis;
    }
    return total;
}

/* out = L u over the whole grid (dimensionless; the Laplacian is Lu / h^2).
 * Returns -1 for an unsupported radius. */
int oracle_laplacian(int R, int64_t nx, int64_t ny, int64_t nz,
                     const double *u, double *out)
{
    double c[9];
    if (oracle_fd_coefficients(R, c) != 0) return -1;
    int64_t z;
#pragma omp parallel for schedule(static)
    for (z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x)
                out[(z * ny + y) * nx + x] = lap_at(R, c, u, nx, ny, nz, z, y, x);
    return 0;
}

/* Leapfrog time loop (Algorithm 1's time loop around the 3D-model step).
 *
 * On entry u_cur = u^{it0}, u_prev = u^{it0-1}. Runs nsteps steps; step n
 * (it0 <= n < it0+nsteps) forms u^{n+1} = 2u^n - u^{n-1} + kappa L u^n and
 * then adds kappa(s_j) * amp[n*nsrc + j] at each source index s_j, in the
 * order j = 0..nsrc-1. On return u_cur = u^{it0+nsteps},
 * u_prev = u^{it0+nsteps-1}. amp must hold at least it0+nsteps rows.
 * Returns 0, or -1 for a bad radius, -2 for a source index outside the grid,
 * -3 when a work buffer cannot be allocated. */
int oracle_leapfrog(int R, int64_t nx, int64_t ny, int64_t nz,
                    const double *kappa, double *u_cur, double *u_prev,
                    int64_t it0, int64_t nsteps,
                    int32_t nsrc, const int64_t *src_idx, const double *amp)
{
    double c[9];
    if (oracle_fd_coefficients(R, c) != 0) return -1;
    const int64_t n = nx * ny * nz;
    for (int32_t j = 0; j < nsrc; ++j)
        if (src_idx[j] < 0 || src_idx[j] >= n) return -2;
    double *next = (double *)malloc((size_t)n * sizeof(double));
    if (!next) return -3;
    for (int64_t step = it0; step < it0 + nsteps; ++step) {
        int64_t z;
#pragma omp parallel for schedule(static)
        for (z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t p = (z * ny + y) * nx + x;
                    next[p] = 2.0 * u_cur[p] - u_prev[p] +
                              kappa[p] * lap_at(R, c, u_cur, nx, ny, nz, z, y, x);
                }
        for (int32_t j = 0; j < nsrc; ++j)
            next[src_idx[j]] += kappa[src_idx[j]] * amp[step * nsrc + j];
        /* rotate: u^{n-1} <- u^n, u^n <- u^{n+1} */
        memcpy(u_prev, u_cur, (size_t)n * sizeof(double));
        memcpy(u_cur, next, (size_t)n * sizeof(double));
    }
    free(next);
    return 0;
}

/* Threads the OpenMP loops use (1 when built without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of later OpenMP loops (n >= 1; no effect without OpenMP). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
