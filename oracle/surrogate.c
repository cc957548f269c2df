/* CPU oracle of the learned k-step surrogate (TEST INFRASTRUCTURE ONLY).
 *
 * The network: four 3x3 convolutions with replicate padding,
 *   2 -> 32 (+GELU) -> 32 (+GELU) -> 32 (+GELU) -> 1,
 * on the normalised inputs t = (T0 - 333)/10, p = (P - 0.5)/0.29; its
 * output y is the normalised k-step increment, T_k = T0 + s*y.
 * GELU is the exact form x Phi(x), Phi(x) = erfc(-x / sqrt 2) / 2 (the normal
 * distribution function; no cancellation for negative x).
 *
 * Everything is evaluated in double.  With round = 1 the operands that the
 * GPU path feeds to its bf16 matrix cores are first rounded to bf16 (round
 * to nearest, ties to even, 8 significant bits): the weights, the network
 * input, the post-GELU activations, and in the backward pass the gradients
 * that enter the weight- and data-gradient products.  Biases, pre-
 * activations, GELU and its derivative, and all sums stay in double.
 *
 * The single convolution and its two adjoints (in the input, in the
 * weights) are exported as well, so that each layer of a GPU evaluation can
 * be checked on its own operands.  OpenMP threads split output channels
 * (input channels for the input adjoint); every sum runs in the same order
 * for any thread count.
 *
 * Weight vector (19393 doubles), canonical order:
 *   W1[32][2][3][3], b1[32], W2[32][32][3][3], b2[32],
 *   W3[32][32][3][3], b3[32], W4[1][32][3][3], b4[1]
 * Image arrays are [H][W] row-major; channel stacks are [C][H][W].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SG_C 32
#define SG_PI 3.14159265358979323846
#define SG_NW 19393

static const int SG_CIN[4] = {2, 32, 32, 32};
static const int SG_COUT[4] = {32, 32, 32, 1};

/* offsets of W_l and b_l in the weight vector */
static void sg_offsets(long wo[4], long bo[4])
{
    long o = 0;
    for (int l = 0; l < 4; ++l) {
        wo[l] = o;
        o += (long)SG_COUT[l] * SG_CIN[l] * 9;
        bo[l] = o;
        o += SG_COUT[l];
    }
}

int or_sg_nweights(void) { return SG_NW; }

/* Round to the nearest bf16 value (8 significant bits), ties to even. */
double or_bf16_round(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    double m = frexp(v, &e);            /* v = m 2^e, 0.5 <= |m| < 1 */
    double r = nearbyint(ldexp(m, 8));  /* 8 significant bits, ties to even */
    return ldexp(r, e - 8);
}

void or_bf16_round_n(const double *v, long n, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = or_bf16_round(v[i]);
}

static double rnd(double v, int round) { return round ? or_bf16_round(v) : v; }

/* Phi, the standard normal distribution function, as erfc(-x/sqrt 2)/2:
 * the same function as (1 + erf(x/sqrt 2))/2 without its cancellation for
 * negative x. */
static double norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

static double gelu(double x) { return x * norm_cdf(x); }

static double gelu_d(double x)
{
    return norm_cdf(x) + x * exp(-0.5 * x * x) / sqrt(2.0 * SG_PI);
}

/* GELU and its derivative elementwise (for checks of a GPU layer's
 * activation and gradient epilogues on the GPU's own pre-activations).   */
void or_sg_gelu(const double *z, long n, double *out, double *dout)
{
    for (long i = 0; i < n; ++i) {
        if (out) out[i] = gelu(z[i]);
        if (dout) dout[i] = gelu_d(z[i]);
    }
}

static long clampi(long v, long n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }

/* out[co][y][x] = b[co] + sum_ci sum_(ky,kx) W[co][ci][ky][kx] *
 *                 in[ci][clamp(y+ky-1)][clamp(x+kx-1)]                    */
void or_sg_conv3x3(const double *W, const double *b, const double *in, int cin, int cout,
                   long H, long Wd, double *out)
{
#pragma omp parallel for schedule(static)
    for (int co = 0; co < cout; ++co)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < Wd; ++x) {
                double acc = b ? b[co] : 0.0;
                for (int ci = 0; ci < cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            acc += W[((co * cin + ci) * 3 + ky) * 3 + kx] *
                                   in[(ci * H + clampi(y + ky - 1, H)) * Wd + clampi(x + kx - 1, Wd)];
                out[(co * H + y) * Wd + x] = acc;
            }
}

/* Adjoint of or_sg_conv3x3 in its input: din[ci][q] = sum over (co, tap,
 * pixel) with clamp(pixel + tap) = q of W[co][ci][tap] * g[co][pixel].
 * Each input channel is accumulated by one thread, in (co, pixel, tap)
 * order.                                                                  */
void or_sg_conv3x3_adjoint_input(const double *W, const double *g, int cin, int cout, long H, long Wd,
                                 double *din)
{
    memset(din, 0, sizeof(double) * cin * H * Wd);
#pragma omp parallel for schedule(static)
    for (int ci = 0; ci < cin; ++ci)
        for (int co = 0; co < cout; ++co)
            for (long y = 0; y < H; ++y)
                for (long x = 0; x < Wd; ++x) {
                    double gv = g[(co * H + y) * Wd + x];
                    if (gv == 0.0) continue;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            din[(ci * H + clampi(y + ky - 1, H)) * Wd + clampi(x + kx - 1, Wd)] +=
                                W[((co * cin + ci) * 3 + ky) * 3 + kx] * gv;
                }
}

/* Gradient in the weights: dW[co][ci][tap] += sum_pixel g[co][pixel] *
 * in[ci][clamp(pixel + tap)], db[co] += sum_pixel gb[co][pixel].        */
void or_sg_conv3x3_adjoint_weights(const double *in, const double *g, const double *gb, int cin, int cout,
                                   long H, long Wd, double *dW, double *db)
{
#pragma omp parallel for schedule(static)
    for (int co = 0; co < cout; ++co)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < Wd; ++x) {
                double gv = g[(co * H + y) * Wd + x];
                db[co] += gb[(co * H + y) * Wd + x];
                for (int ci = 0; ci < cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            dW[((co * cin + ci) * 3 + ky) * 3 + kx] +=
                                gv * in[(ci * H + clampi(y + ky - 1, H)) * Wd + clampi(x + kx - 1, Wd)];
            }
}

typedef struct {
    double *x;          /* [2][H][W] network input (rounded if round)     */
    double *z[4];       /* pre-activations of layers 1..4                   */
    double *a[3];       /* post-GELU activations of layers 1..3 (rounded) */
    double *w;          /* weights as used (rounded if round)              */
} sg_tape;

static void tape_free(sg_tape *t)
{
    free(t->x); free(t->w);
    for (int l = 0; l < 4; ++l) free(t->z[l]);
    for (int l = 0; l < 3; ++l) free(t->a[l]);
}

static int forward(const double *w_in, const float *T0, const float *P, long H, long Wd, int round, sg_tape *t)
{
    long n = H * Wd, wo[4], bo[4];
    sg_offsets(wo, bo);
    memset(t, 0, sizeof(*t));
    t->x = malloc(sizeof(double) * 2 * n);
    t->w = malloc(sizeof(double) * SG_NW);
    for (int l = 0; l < 4; ++l) t->z[l] = malloc(sizeof(double) * SG_COUT[l] * n);
    for (int l = 0; l < 3; ++l) t->a[l] = malloc(sizeof(double) * SG_C * n);
    if (!t->x || !t->w || !t->z[3] || !t->a[2]) { tape_free(t); return -1; }
    for (long i = 0; i < SG_NW; ++i) t->w[i] = w_in[i];
    for (int l = 0; l < 4; ++l)
        for (long i = 0; i < (long)SG_COUT[l] * SG_CIN[l] * 9; ++i) t->w[wo[l] + i] = rnd(w_in[wo[l] + i], round);
    for (long i = 0; i < n; ++i) {
        t->x[i] = rnd(((double)T0[i] - 333.0) / 10.0, round);
        t->x[n + i] = rnd(((double)P[i] - 0.5) / 0.29, round);
    }
    const double *in = t->x;
    for (int l = 0; l < 4; ++l) {
        or_sg_conv3x3(t->w + wo[l], t->w + bo[l], in, SG_CIN[l], SG_COUT[l], H, Wd, t->z[l]);
        if (l < 3) {
            for (long i = 0; i < SG_C * n; ++i) t->a[l][i] = rnd(gelu(t->z[l][i]), round);
            in = t->a[l];
        }
    }
    return 0;
}

/* Network output y[H][W] (the normalised k-step increment). */
int or_sg_forward(const double *w, const float *T0, const float *P, long H, long Wd, int round, double *y)
{
    sg_tape t;
    if (forward(w, T0, P, H, Wd, round, &t)) return -1;
    memcpy(y, t.z[3], sizeof(double) * H * Wd);
    tape_free(&t);
    return 0;
}

/* Loss L = sum_pixels (y - target)^2 / norm and its gradient dL/dw
 * (accumulated into grad, which the caller zeroes).  norm is the number of
 * pixels the caller averages over (e.g. batch * H * W).                    */
int or_sg_loss_grad(const double *w, const float *T0, const float *P, const double *target, long H, long Wd,
                    double norm, int round, double *grad, double *loss)
{
    long n = H * Wd, wo[4], bo[4];
    sg_offsets(wo, bo);
    sg_tape t;
    if (forward(w, T0, P, H, Wd, round, &t)) return -1;
    double *g = malloc(sizeof(double) * SG_C * n);    /* gradient entering a product */
    double *gb = malloc(sizeof(double) * SG_C * n);   /* unrounded, for the bias     */
    double *da = malloc(sizeof(double) * SG_C * n);
    if (!g || !gb || !da) { free(g); free(gb); free(da); tape_free(&t); return -1; }
    double L = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = t.z[3][i] - target[i];
        L += d * d;
        gb[i] = 2.0 * d / norm;
        g[i] = rnd(gb[i], round);
    }
    *loss = L / norm;
    for (int l = 3; l >= 0; --l) {
        const double *in = l == 0 ? t.x : t.a[l - 1];
        or_sg_conv3x3_adjoint_weights(in, g, gb, SG_CIN[l], SG_COUT[l], H, Wd, grad + wo[l], grad + bo[l]);
        if (l == 0) break;
        or_sg_conv3x3_adjoint_input(t.w + wo[l], g, SG_CIN[l], SG_COUT[l], H, Wd, da);
        for (long i = 0; i < SG_C * n; ++i) {
            gb[i] = da[i] * gelu_d(t.z[l - 1][i]);
            g[i] = rnd(gb[i], round);
        }
    }
    free(g); free(gb); free(da);
    tape_free(&t);
    return 0;
}

/* One Adam step (Kingma and Ba 2015) at step count ts >= 1, in place:
 * m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * w -= lr * (m / (1 - b1^ts)) / (sqrt(v / (1 - b2^ts)) + eps).         */
void or_adam(double *w, const double *g, double *m, double *v, long n, long ts, double lr, double b1, double b2,
             double eps)
{
    double c1 = 1.0 - pow(b1, (double)ts), c2 = 1.0 - pow(b2, (double)ts);
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
