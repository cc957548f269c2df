/* CPU oracle for the iterative solvers that the batching method drives.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU product
 * path never calls it, and it shares no source with the GPU library.
 *
 * Each solver is instantiated twice from oracle_impl.h: in float (the
 * precision of the GPU path) and in double (the accuracy reference).
 * What each function follows:
 *   or_heat2d_*    the explicit 2D thermal update (Hotspot, Sec. III-C)
 *   or_heat3d_*    the layered 3D thermal update (Hotspot3D, Sec. III-C)
 *   or_skeleton_*  the skeleton application's chain of small kernels
 *                  (Sec. III-C), generalised to x <- a_k*x + b_k
 *   or_fdtd_*      the FDTD Maxwell cavity solver (Sec. III-C): H, E, source
 *   or_fdtd_pulse  the soft-source amplitude table
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define REAL float
#define SFX(name) name##_f32
#define SKEL_AXPB(a, x, b) fmaf((a), (x), (b))
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef SKEL_AXPB

#define REAL double
#define SFX(name) name##_f64
#define SKEL_AXPB(a, x, b) ((a) * (x) + (b))
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef SKEL_AXPB

/* Gaussian soft-source amplitude per absolute step n:
 *   g(n) = exp(-((n - n0)/w)^2), evaluated in double.
 * g64 (may be NULL) receives the double values, g32 (may be NULL) the same
 * values rounded once to float.                                           */
void or_fdtd_pulse(double n0, double w, long count, double *g64, float *g32)
{
    for (long n = 0; n < count; ++n) {
        double x = ((double)n - n0) / w;
        double v = exp(-(x * x));
        if (g64) g64[n] = v;
        if (g32) g32[n] = (float)v;
    }
}

/* Threads of the loops that split independent rows, planes or elements
 * (n >= 1; the results are the same bits for every n).                   */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }

int or_abi_version(void) { return 2; }
