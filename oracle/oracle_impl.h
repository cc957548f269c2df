/* Body of the CPU oracle, written once and instantiated for float and for
 * double by oracle.c (REAL = element type, SFX(name) = name_f32 / name_f64).
 *
 * This is test infrastructure: a plain, slow, obviously correct statement
 * of what the solvers compute, used only by the tests, by the smoke check
 * and by the CPU-baseline leg of the benchmark.  It shares no code with the
 * GPU library.  Every loop follows the definition it cites; there is no
 * blocking, fusion or reordering beyond that definition.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp, so that no multiply-add is
 * fused unless the source calls fma explicitly.  OpenMP threads only split
 * loops whose iterations are independent (rows, planes, elements); every
 * value is computed by the same operations in the same order whatever the
 * thread count, so the results do not depend on it (or_set_threads).
 */

/* ------------------------------------------------------------------------ */
/* 2D thermal stencil (Hotspot-style model, Sec. III-C; update of the       */
/* 256x256 workload): per step, with neighbour indices clamped to the grid, */
/*   T' = T + c*(P + (Tn+Ts-2T)/Ry + (Te+Tw-2T)/Rx + (Tamb-T)/Rz).          */
/* n/s are rows i-1/i+1 (paired with Ry), w/e are columns j-1/j+1 (Rx).      */
/* The expression is evaluated left to right exactly as written.            */
/* ------------------------------------------------------------------------ */
static void SFX(heat2d_step)(const REAL *T, const REAL *P, REAL *out,
                             long ny, long nx, REAL c, REAL Rx, REAL Ry,
                             REAL Rz, REAL Tamb)
{
    /* rows are independent within a step (threads only split the rows) */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < ny; ++i) {
        long in = i > 0 ? i - 1 : 0;
        long is = i < ny - 1 ? i + 1 : ny - 1;
        for (long j = 0; j < nx; ++j) {
            long jw = j > 0 ? j - 1 : 0;
            long je = j < nx - 1 ? j + 1 : nx - 1;
            REAL t = T[i * nx + j];
            REAL tn = T[in * nx + j], ts = T[is * nx + j];
            REAL tw = T[i * nx + jw], te = T[i * nx + je];
            REAL p = P[i * nx + j];
            out[i * nx + j] = t + c * (p + (tn + ts - 2 * t) / Ry
                                         + (te + tw - 2 * t) / Rx
                                         + (Tamb - t) / Rz);
        }
    }
}

/* Advance T0 by nsteps steps; result in out (ny*nx). Ping-pong buffers. */
int SFX(or_heat2d)(const REAL *T0, const REAL *P, long ny, long nx,
                   double c, double Rx, double Ry, double Rz, double Tamb,
                   long nsteps, REAL *out)
{
    long n = ny * nx;
    REAL *a = (REAL *)malloc(sizeof(REAL) * n);
    REAL *b = (REAL *)malloc(sizeof(REAL) * n);
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, T0, sizeof(REAL) * n);
    for (long s = 0; s < nsteps; ++s) {
        SFX(heat2d_step)(a, P, b, ny, nx, (REAL)c, (REAL)Rx, (REAL)Ry,
                         (REAL)Rz, (REAL)Tamb);
        REAL *t = a; a = b; b = t;
    }
    memcpy(out, a, sizeof(REAL) * n);
    free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3D thermal stencil (Hotspot3D-style layered model): the 2D update plus   */
/* the vertical term (Tu+Td-2T)/Rz with clamped layer index; the ambient     */
/* term applies on every layer; P is given per cell (dense nz*ny*nx).        */
/* Layout [z][y][x], x fastest.                                              */
/* ------------------------------------------------------------------------ */
static void SFX(heat3d_step)(const REAL *T, const REAL *P, REAL *out,
                             long nz, long ny, long nx, REAL c, REAL Rx,
                             REAL Ry, REAL Rz, REAL Tamb)
{
    long plane = ny * nx;
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z) {
        for (long i = 0; i < ny; ++i) {
            long zd = z > 0 ? z - 1 : 0;
            long zu = z < nz - 1 ? z + 1 : nz - 1;
            long in = i > 0 ? i - 1 : 0;
            long is = i < ny - 1 ? i + 1 : ny - 1;
            for (long j = 0; j < nx; ++j) {
                long jw = j > 0 ? j - 1 : 0;
                long je = j < nx - 1 ? j + 1 : nx - 1;
                long o = z * plane + i * nx + j;
                REAL t = T[o];
                REAL tn = T[z * plane + in * nx + j];
                REAL ts = T[z * plane + is * nx + j];
                REAL tw = T[z * plane + i * nx + jw];
                REAL te = T[z * plane + i * nx + je];
                REAL tu = T[zu * plane + i * nx + j];
                REAL td = T[zd * plane + i * nx + j];
                out[o] = t + c * (P[o] + (tn + ts - 2 * t) / Ry
                                       + (te + tw - 2 * t) / Rx
                                       + (tu + td - 2 * t) / Rz
                                       + (Tamb - t) / Rz);
            }
        }
    }
}

int SFX(or_heat3d)(const REAL *T0, const REAL *P, long nz, long ny, long nx,
                   double c, double Rx, double Ry, double Rz, double Tamb,
                   long nsteps, REAL *out)
{
    long n = nz * ny * nx;
    REAL *a = (REAL *)malloc(sizeof(REAL) * n);
    REAL *b = (REAL *)malloc(sizeof(REAL) * n);
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, T0, sizeof(REAL) * n);
    for (long s = 0; s < nsteps; ++s) {
        SFX(heat3d_step)(a, P, b, nz, ny, nx, (REAL)c, (REAL)Rx, (REAL)Ry,
                         (REAL)Rz, (REAL)Tamb);
        REAL *t = a; a = b; b = t;
    }
    memcpy(out, a, sizeof(REAL) * n);
    free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Skeleton iterative application (Sec. III-C): each iteration runs K small */
/* element-wise kernels in order, kernel k computing x <- a_k*x + b_k.       */
/* The float version rounds once per kernel (fused multiply-add); the       */
/* double version is the plain product-then-sum.                            */
/* ------------------------------------------------------------------------ */
int SFX(or_skeleton)(const REAL *x0, long n, const REAL *a, const REAL *b,
                     int K, long iters, REAL *out)
{
    /* every element runs its own chain: iteration by iteration, kernel by
     * kernel, the same operations as the kernel-major loop of the method */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e) {
        REAL x = x0[e];
        for (long it = 0; it < iters; ++it)
            for (int k = 0; k < K; ++k)
                x = SKEL_AXPB(a[k], x, b[k]);
        out[e] = x;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* FDTD Maxwell solver for a PEC cavity (Sec. III-C): Yee leapfrog with      */
/* dx = 1, eps = mu = 1.  Every field is stored on a padded (N+1)^3 grid,     */
/* index (k*(N+1)+j)*(N+1)+i.  Component positions:                          */
/*   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)                   */
/*   Hx (i, j+1/2, k+1/2)  Hy (i+1/2, j, k+1/2)  Hz (i+1/2, j+1/2, k)          */
/* One step: (1) H -= dt*curl E on every H node; (2) E += dt*curl H on the  */
/* interior E nodes only (tangential E on the walls stays zero: PEC);       */
/* (3) Ez at the source node += g(n), then the probe records that Ez.       */
/* ------------------------------------------------------------------------ */
#define FX(a, i, j, k) (a)[((long)(k) * M + (j)) * M + (i)]

static void SFX(fdtd_h)(REAL *Hx, REAL *Hy, REAL *Hz, const REAL *Ex,
                        const REAL *Ey, const REAL *Ez, long N, REAL dt)
{
    long M = N + 1;
    /* each H node reads only E: the planes are independent */
#pragma omp parallel for schedule(static)
    for (long k = 0; k <= N; ++k)
        for (long j = 0; j <= N; ++j)
            for (long i = 0; i <= N; ++i) {
                if (j < N && k < N)  /* Hx: dEz/dy - dEy/dz */
                    FX(Hx, i, j, k) -= dt * ((FX(Ez, i, j + 1, k) - FX(Ez, i, j, k))
                                           - (FX(Ey, i, j, k + 1) - FX(Ey, i, j, k)));
                if (i < N && k < N)  /* Hy: dEx/dz - dEz/dx */
                    FX(Hy, i, j, k) -= dt * ((FX(Ex, i, j, k + 1) - FX(Ex, i, j, k))
                                           - (FX(Ez, i + 1, j, k) - FX(Ez, i, j, k)));
                if (i < N && j < N)  /* Hz: dEy/dx - dEx/dy */
                    FX(Hz, i, j, k) -= dt * ((FX(Ey, i + 1, j, k) - FX(Ey, i, j, k))
                                           - (FX(Ex, i, j + 1, k) - FX(Ex, i, j, k)));
            }
}

static void SFX(fdtd_e)(REAL *Ex, REAL *Ey, REAL *Ez, const REAL *Hx,
                        const REAL *Hy, const REAL *Hz, long N, REAL dt)
{
    long M = N + 1;
    /* each E node reads only H: the planes are independent */
#pragma omp parallel for schedule(static)
    for (long k = 0; k <= N; ++k)
        for (long j = 0; j <= N; ++j)
            for (long i = 0; i <= N; ++i) {
                int ii = i >= 1 && i <= N - 1;
                int jj = j >= 1 && j <= N - 1;
                int kk = k >= 1 && k <= N - 1;
                if (i < N && jj && kk)  /* Ex: dHz/dy - dHy/dz */
                    FX(Ex, i, j, k) += dt * ((FX(Hz, i, j, k) - FX(Hz, i, j - 1, k))
                                           - (FX(Hy, i, j, k) - FX(Hy, i, j, k - 1)));
                if (j < N && ii && kk)  /* Ey: dHx/dz - dHz/dx */
                    FX(Ey, i, j, k) += dt * ((FX(Hx, i, j, k) - FX(Hx, i, j, k - 1))
                                           - (FX(Hz, i, j, k) - FX(Hz, i - 1, j, k)));
                if (k < N && ii && jj)  /* Ez: dHy/dx - dHx/dy */
                    FX(Ez, i, j, k) += dt * ((FX(Hy, i, j, k) - FX(Hy, i - 1, j, k))
                                           - (FX(Hx, i, j, k) - FX(Hx, i, j - 1, k)));
            }
}

/* Advance the six fields (each (N+1)^3, updated in place) by nsteps steps,
 * starting at absolute step n_start.  src = {i, j, k} of the Ez source node,
 * g = source amplitude per absolute step (length >= n_start + nsteps) or
 * NULL for no source.  probe (length nsteps, may be NULL) receives Ez at the
 * source node after each step.  Fields order: Ex, Ey, Ez, Hx, Hy, Hz.       */
int SFX(or_fdtd)(REAL *Ex, REAL *Ey, REAL *Ez, REAL *Hx, REAL *Hy, REAL *Hz,
                 long N, double dt, const long *src, const REAL *g,
                 long n_start, long nsteps, REAL *probe)
{
    long M = N + 1;
    for (long s = 0; s < nsteps; ++s) {
        SFX(fdtd_h)(Hx, Hy, Hz, Ex, Ey, Ez, N, (REAL)dt);
        SFX(fdtd_e)(Ex, Ey, Ez, Hx, Hy, Hz, N, (REAL)dt);
        if (g) FX(Ez, src[0], src[1], src[2]) += g[n_start + s];
        if (probe) probe[s] = FX(Ez, src[0], src[1], src[2]);
    }
    return 0;
}

#undef FX
