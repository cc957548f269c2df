// Learned k-step surrogate of the 2D thermal stencil: kernels.
//
// Network: four 3x3 convolutions with replicate padding,
//   2 -> 32 (+GELU) -> 32 (+GELU) -> 32 (+GELU) -> 1,
// on t = (T0 - 333)/10 and p = (P - 0.5)/0.29; the output y is the
// normalised k-step increment and T_k = T0 + s*y (float32 add).
//
// The convolutions are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16: A 16x32, B 32x16, D 16x16 float32).  Lane l of
// a wave holds A row l%16 and B column l%16 at k = (l/16)*8 .. +7, and D
// column l%16 at rows (l/16)*4 .. +3.
//   forward : D[cout][pixel]   = sum_(tap,cin)  W[cout][cin][tap] x[src(pixel,tap)][cin]
//   dgrad   : D[cin][pixel]    = sum_(tap,cout) W[cout][cin][tap] g~[tap][cout][pixel]
//             where g~ sums the upstream gradient over every pixel whose
//             clamped tap lands on `pixel` (the adjoint of replicate padding)
//   wgrad   : D[cout][(tap,cin)] = sum_pixel g[pixel][cout] x[src(pixel,tap)][cin]
// Activations are stored pixel-major (channels contiguous, 64 bytes per
// pixel in bf16) so a lane's 8-channel fragment is one 16-byte load.
// Operands are rounded to bf16 (nearest, ties to even) exactly where the
// oracle rounds them; accumulation is float32; biases, GELU and its
// derivative are float32.  Reductions over pixels (weight and bias
// gradients, loss) go through per-block partials summed in a fixed order,
// so every result is deterministic.
#include "heat_update.h"
#include "kb_internal.h"
#include "sg_internal.h"

namespace kb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// float -> bf16 bits, round to nearest, ties to even (the hardware
// conversion, v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned f2bf2(float a, float b) {
  const bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ bf16x8 ld_frag(const unsigned short *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}
__device__ __forceinline__ bf16x8 make_frag(const unsigned short (&v)[8]) {
  u16x8 u = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// GELU(x) = x Phi(x), Phi the standard normal distribution function, and
// GELU'(x) = Phi(x) + x phi(x).  Phi(x) = erfc(-x / sqrt 2) / 2 is evaluated
// so that it keeps its relative accuracy for negative x, where
// (1 + erf(x / sqrt 2)) / 2 would cancel:
//   |x| <= 1: Phi = 1/2 + x S(x^2), S a degree-5 polynomial;
//   |x| >  1: erfc(v) = exp(-v^2) R(v), v = |x| / sqrt 2, R the scaled
//             complementary error function as a (4, 5) rational function
//             fitted on [0, 10]; exp(-x^2 / 2) = 2^(-x^2 log2(e) / 2) with
//             x^2 and the product carried to about twice float32 precision
//             (an error in the exponent would be amplified by x^2).
// Phi = erfc/2 for x < 0 and 1 - erfc/2 for x > 0.  Coefficients: minimax
// fits in relative error (gelu_coeffs.py).  Error, in float32 arithmetic:
// at most about 8 units of 2^-24 relative (mean 1) over [-13, 8]; below
// x = -13 the exponential leaves the normal float range and GELU returns -0.
// The polynomial piece runs for the lanes with |x| <= 1, the rest only where
// a lane of the wave needs it.
constexpr float kPhiS[6] = {3.989422917e-01f, -6.649035960e-02f, 9.973322973e-03f, -1.186329755e-03f, 1.134861304e-04f, -7.654097317e-06f};
constexpr float kErfcxP[5] = {1.000000000e+00f, 1.237535715e+00f, 7.306861281e-01f, 2.287804782e-01f, 3.270421550e-02f};
constexpr float kErfcxQ[6] = {1.000000000e+00f, 2.365915537e+00f, 2.400326729e+00f, 1.323654652e+00f, 4.055296779e-01f, 5.796599761e-02f};

__device__ __forceinline__ float norm_cdf_tail(float x) {
  constexpr float kC = 0.7213475108146667f;                  // log2(e) / 2, rounded to float
  constexpr float kCl = 9.62981494545545e-09f;               // log2(e) / 2 - kC
  constexpr float kLn2 = 0.6931471805599453f;
  const float sq = x * x, se = fmaf(x, x, -sq);               // x^2 = sq + se exactly
  const float yh = sq * kC;
  const float yl = fmaf(se, kC, fmaf(sq, kCl, fmaf(sq, kC, -yh)));
  const float e2 = __builtin_amdgcn_exp2f(-yh);
  const float ex = fmaf(e2, -yl * kLn2, e2);                  // exp(-x^2 / 2)
  const float v = fabsf(x) * 0.70710678118654752f;
  float p = kErfcxP[4], q = kErfcxQ[5];
#pragma unroll
  for (int i = 3; i >= 0; --i) p = fmaf(p, v, kErfcxP[i]);
#pragma unroll
  for (int i = 4; i >= 0; --i) q = fmaf(q, v, kErfcxQ[i]);
  const float rq = __builtin_amdgcn_rcpf(q);
  float R = p * rq;
  R = fmaf(fmaf(-q, R, p), rq, R);                            // one correction of the quotient
  const float E = ex * R;                                     // erfc(v)
  return x < 0.f ? 0.5f * E : fmaf(-0.5f, E, 1.0f);
}
__device__ __forceinline__ float norm_cdf(float x) {
  if (fabsf(x) <= 1.0f) {
    const float w = x * x;
    float s = kPhiS[5];
#pragma unroll
    for (int i = 4; i >= 0; --i) s = fmaf(s, w, kPhiS[i]);
    return fmaf(x, s, 0.5f);
  }
  return norm_cdf_tail(x);
}
__device__ __forceinline__ float gelu(float x) { return x * norm_cdf(x); }
__device__ __forceinline__ float gelu_d(float x) {
  return norm_cdf(x) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }

struct Pix {
  int img, y, x;
};
__device__ __forceinline__ Pix pix_of(long long p, int H, int W) {
  Pix r;
  const long long hw = (long long)H * W;
  r.img = (int)(p / hw);
  const int rem = (int)(p - (long long)r.img * hw);
  r.y = rem / W;
  r.x = rem - r.y * W;
  return r;
}
__device__ __forceinline__ long long pix_at(const Pix &q, int y, int x, int H, int W) {
  return ((long long)q.img * H + y) * W + x;
}

// ---------------------------------------------------------------------------
// Network input: x[p] = (bf16((T0-333)/10), bf16((P-0.5)/0.29)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sg_input_kernel(const SgInputArgs a) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= a.npix) return;
  const float t = (a.T0[p] - 333.0f) / 10.0f;
  const float q = (a.P[p] - 0.5f) / 0.29f;
  const unsigned v = (unsigned)f2bf(t) | ((unsigned)f2bf(q) << 16);
  reinterpret_cast<unsigned *>(a.x)[p] = v;
}

// ---------------------------------------------------------------------------
// Forward convolution.  A wave computes all output channels for 64 pixels
// (four groups of 16); a block is four waves (256 pixels).
//   CIN = 2 : one K block, k = tap*2 + cin (18 used, 14 zero).
//   CIN = 32: nine K blocks (one per tap), k = cin.
//   COUT = 32: D rows are channels (two 16-row tiles); epilogue adds the
//              bias, optionally stores z (float32), stores bf16(GELU(z)).
//   COUT = 1 : one tile whose row 0 is the channel (rows 1..15 zero);
//              epilogue stores y = z and, for inference, T0 + s*y.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void sg_conv_fwd_kernel(const SgConvArgs a) {
  constexpr int MT = COUT == 32 ? 2 : 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long base = ((long long)blockIdx.x * 4 + wave) * 64;
  if (base >= a.npix) return;
  const int r = lane & 15, kq = lane >> 4;
  Pix pg[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    long long p = base + g * 16 + r;
    if (p >= a.npix) p = a.npix - 1;
    pg[g] = pix_of(p, a.H, a.W);
  }
  // 32-channel layers start the accumulator at the bias (the fused kernel
  // does the same, so both give the same hidden activations)
  f32x4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g)
      acc[m][g] = COUT == 32 ? *reinterpret_cast<const f32x4 *>(a.bias + m * 16 + kq * 4) : f32x4{0.f, 0.f, 0.f, 0.f};

  if constexpr (CIN == 32) {
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      bf16x8 A[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (COUT == 32 || r == 0)
          A[m] = ld_frag(a.w + ((size_t)(tap * (COUT == 32 ? 32 : 1) + (COUT == 32 ? m * 16 + r : 0)) * 32 + kq * 8));
        else
          A[m] = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const long long src = pix_at(pg[g], clampi(pg[g].y + dy, a.H), clampi(pg[g].x + dx, a.W), a.H, a.W);
        const bf16x8 B = ld_frag(a.in + src * 32 + kq * 8);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][g] = mfma(A[m], B, acc[m][g]);
      }
    }
  } else {
    bf16x8 A[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) A[m] = ld_frag(a.w + (size_t)(m * 16 + r) * 32 + kq * 8);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      unsigned short v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kq * 8 + i;
        v[i] = 0;
        if (k < 18) {
          const int tap = k >> 1, ci = k & 1;
          const long long src =
              pix_at(pg[g], clampi(pg[g].y + tap / 3 - 1, a.H), clampi(pg[g].x + tap % 3 - 1, a.W), a.H, a.W);
          v[i] = a.in[src * 2 + ci];
        }
      }
      const bf16x8 B = make_frag(v);
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m][g] = mfma(A[m], B, acc[m][g]);
    }
  }

#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const long long p = base + g * 16 + r;
    if (p >= a.npix) continue;
    if constexpr (COUT == 32) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int c0 = m * 16 + kq * 4;
        float z[4];
        unsigned short h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          z[j] = acc[m][g][j];
          h[j] = f2bf(gelu(z[j]));
        }
        if (a.z) *reinterpret_cast<float4 *>(a.z + p * 32 + c0) = make_float4(z[0], z[1], z[2], z[3]);
        uint2 packed;
        packed.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
        packed.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
        *reinterpret_cast<uint2 *>(a.out + p * 32 + c0) = packed;
      }
    } else {
      if (kq == 0) {
        const float y = acc[0][g][0] + a.bias[0];
        if (a.y) a.y[p] = y;
        if (a.Tout) a.Tout[p] = a.T0[p] + a.s * y;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Loss: g4 = 2 (y - target) / norm per pixel; per-block partial sums of
// (y - target)^2 in double.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double v, double *sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void sg_loss_kernel(const SgLossArgs a) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.npix; p += (long long)gridDim.x * 256) {
    const float d = a.y[p] - a.target[p];
    a.g[p] = 2.0f * d / a.norm;
    acc += (double)d * (double)d;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Data gradient of layer l (COUT = its output channels, 32 or 1) into the
// 32 channels of its input, times GELU'(z_{l-1}):
//   gout[q][cin] = gelu'(z[q][cin]) * sum_(tap, cout) W[cout][cin][tap] *
//                  sum_{p : clamp(p + tap) = q} bf16(g[p][cout])
// The inner sum over source pixels has one term away from the edges and up
// to four at an image corner.  Each source pixel enters the matrix cores as
// its own bf16 operand (one MFMA per source slot), so every product is exact
// and only float32 sums follow, as in the convolution's other products;
// slots beyond the first run only where a lane of the wave lies on an edge.
// ---------------------------------------------------------------------------
// Pixels p along one axis with clamp(p + d) == q (at most two).
__device__ __forceinline__ int adj_src(int q, int d, int n, int *out) {
  int c = 0;
#pragma unroll
  for (int s = -1; s <= 1; ++s) {
    const int p = q - d + s;
    if (p >= 0 && p < n && clampi(p + d, n) == q) out[c++] = p;
  }
  return c;
}

template <int COUT>
__global__ __launch_bounds__(256) void sg_dgrad_kernel(const SgDgradArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long base = ((long long)blockIdx.x * 4 + wave) * 64;
  if (base >= a.npix) return;
  const int r = lane & 15, kq = lane >> 4;
  Pix pg[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    long long p = base + g * 16 + r;
    if (p >= a.npix) p = a.npix - 1;
    pg[g] = pix_of(p, a.H, a.W);
  }
  f32x4 acc[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[m][g] = f32x4{0.f, 0.f, 0.f, 0.f};

  if constexpr (COUT == 32) {
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      bf16x8 A[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) A[m] = ld_frag(a.w + ((size_t)(tap * 32 + m * 16 + r)) * 32 + kq * 8);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        int ys[3], xs[3];
        const int ny = adj_src(pg[g].y, dy, a.H, ys);
        const int nx = adj_src(pg[g].x, dx, a.W, xs);
        const int ns = ny * nx;
        for (int k = 0; k < 4; ++k) {
          if (k > 0 && !__any(k < ns)) break;          // wave-uniform
          unsigned short v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          if (k < ns) {
            const float *gp = a.g + pix_at(pg[g], ys[k / nx], xs[k % nx], a.H, a.W) * 32 + kq * 8;
            const float4 v0 = *reinterpret_cast<const float4 *>(gp);
            const float4 v1 = *reinterpret_cast<const float4 *>(gp + 4);
            v[0] = f2bf(v0.x); v[1] = f2bf(v0.y); v[2] = f2bf(v0.z); v[3] = f2bf(v0.w);
            v[4] = f2bf(v1.x); v[5] = f2bf(v1.y); v[6] = f2bf(v1.z); v[7] = f2bf(v1.w);
          }
          const bf16x8 B = make_frag(v);
#pragma unroll
          for (int m = 0; m < 2; ++m) acc[m][g] = mfma(A[m], B, acc[m][g]);
        }
      }
    }
  } else {
    bf16x8 A[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) A[m] = ld_frag(a.w + (size_t)(m * 16 + r) * 32 + kq * 8);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      // K runs over the taps (kq*8 + i < 9); slot k of tap i is its k-th
      // source pixel
      int nmax = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int tap = kq * 8 + i;
        if (tap < 9) {
          int ys[3], xs[3];
          const int ns = adj_src(pg[g].y, tap / 3 - 1, a.H, ys) * adj_src(pg[g].x, tap % 3 - 1, a.W, xs);
          nmax = ns > nmax ? ns : nmax;
        }
      }
      for (int k = 0; k < 4; ++k) {
        if (k > 0 && !__any(k < nmax)) break;          // wave-uniform
        unsigned short v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int tap = kq * 8 + i;
          float val = 0.f;
          if (tap < 9) {
            int ys[3], xs[3];
            const int ny = adj_src(pg[g].y, tap / 3 - 1, a.H, ys);
            const int nx = adj_src(pg[g].x, tap % 3 - 1, a.W, xs);
            if (k < ny * nx) val = a.g[pix_at(pg[g], ys[k / nx], xs[k % nx], a.H, a.W)];
          }
          v[i] = f2bf(val);
        }
        const bf16x8 B = make_frag(v);
#pragma unroll
        for (int m = 0; m < 2; ++m) acc[m][g] = mfma(A[m], B, acc[m][g]);
      }
    }
  }

#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const long long p = base + g * 16 + r;
    if (p >= a.npix) continue;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int c0 = m * 16 + kq * 4;
      const float4 z = *reinterpret_cast<const float4 *>(a.z + p * 32 + c0);
      float4 o;
      o.x = acc[m][g][0] * gelu_d(z.x);
      o.y = acc[m][g][1] * gelu_d(z.y);
      o.z = acc[m][g][2] * gelu_d(z.z);
      o.w = acc[m][g][3] * gelu_d(z.w);
      *reinterpret_cast<float4 *>(a.gout + p * 32 + c0) = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of one layer: per block, partial sums over a fixed range
// of row segments of 64 pixels (W must be a multiple of 64):
//   dW[cout][tap*CIN + cin] = sum_p bf16(g[p][cout]) * x[src(p, tap)][cin]
//   db[cout]                = sum_p g[p][cout]            (float32 g)
// The segment's gradient (transposed, rounded) and the three input rows it
// touches (with one clamped column on each side) are staged in LDS.  The
// GEMM has M = COUT (two tiles, or one padded tile for COUT = 1), N =
// 9*CIN columns (18 tiles, or 2 for CIN = 2) split over the four waves, and
// K = the 64 pixels (two K blocks).
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void sg_wgrad_kernel(const SgWgradArgs a) {
  constexpr int MT = COUT == 32 ? 2 : 1;
  constexpr int NCOL = 9 * CIN;
  constexpr int NT = (NCOL + 15) / 16;
  constexpr int NTW = (NT + 3) / 4;        // column tiles per wave
  constexpr int GR = COUT == 32 ? 32 : 16; // rows of the staged gradient
  __shared__ unsigned short gs[GR][64 + 8];
  __shared__ unsigned short xs[3][66][CIN];
  __shared__ double dsh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int segs_per_row = a.W / 64;
  const long long nseg = (long long)a.nimg * a.H * segs_per_row;
  const long long s0 = nseg * blockIdx.x / gridDim.x, s1 = nseg * (blockIdx.x + 1) / gridDim.x;

  f32x4 acc[MT][NTW];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;   // bias partial of channel threadIdx.x (< COUT)

  for (long long sg = s0; sg < s1; ++sg) {
    const int img = (int)(sg / ((long long)a.H * segs_per_row));
    const int rem = (int)(sg - (long long)img * a.H * segs_per_row);
    const int y = rem / segs_per_row, x0 = (rem - y * segs_per_row) * 64;
    const long long p0 = ((long long)img * a.H + y) * a.W + x0;
    // stage the gradient: gs[cout][px] = bf16(g[p0+px][cout]); bias sums
    for (int e = threadIdx.x; e < 64 * COUT; e += 256) {
      const int px = e / COUT, c = e - px * COUT;
      const float gv = a.g[(p0 + px) * COUT + c];
      gs[c][px] = f2bf(gv);
    }
    if (COUT == 1)
      for (int e = threadIdx.x; e < 15 * 64; e += 256) gs[1 + e / 64][e % 64] = 0;
    if (threadIdx.x < COUT)
      for (int px = 0; px < 64; ++px) bsum += a.g[(p0 + px) * COUT + threadIdx.x];
    // stage the input rows y-1, y, y+1 at columns x0-1 .. x0+64 (clamped)
    for (int e = threadIdx.x; e < 3 * 66 * CIN; e += 256) {
      const int rr = e / (66 * CIN), rem2 = e - rr * 66 * CIN;
      const int cc = rem2 / CIN, ci = rem2 - cc * CIN;
      const int yy = clampi(y + rr - 1, a.H), xx = clampi(x0 + cc - 1, a.W);
      xs[rr][cc][ci] = a.x[(((long long)img * a.H + yy) * a.W + xx) * CIN + ci];
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int pxb = kb * 32 + kq * 8;
      bf16x8 A[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        unsigned short v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = gs[m * 16 + r][pxb + i];
        A[m] = make_frag(v);
      }
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int tile = wave + 4 * t;
        if (tile >= NT) break;
        const int col = tile * 16 + r;
        unsigned short v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (col < NCOL) {
          const int tap = col / CIN, ci = col - tap * CIN;
          const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = xs[1 + dy][1 + pxb + i + dx][ci];
        }
        const bf16x8 B = make_frag(v);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][t] = mfma(A[m], B, acc[m][t]);
      }
    }
    __syncthreads();
  }
  // partial dW: rows = cout, columns = tap*CIN + cin
  float *pw = a.partial_w + (size_t)blockIdx.x * COUT * NCOL;
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= NT) break;
    const int col = tile * 16 + r;
    if (col >= NCOL) continue;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = m * 16 + kq * 4 + j;
        if (co < COUT) pw[co * NCOL + col] = acc[m][t][j];
      }
  }
  if (threadIdx.x < COUT) a.partial_b[(size_t)blockIdx.x * COUT + threadIdx.x] = bsum;
  (void)dsh;
}

// Sum the per-block partials in block order into the canonical gradient:
// W[cout][cin][ky][kx] (tap = ky*3 + kx) and b[cout].
__global__ __launch_bounds__(256) void sg_grad_reduce_kernel(const SgReduceArgs a) {
  const int ncol = 9 * a.cin;
  const int nw = a.cout * ncol;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < nw) {
    float s = 0.f;
    for (int b = 0; b < a.nblk; ++b) s += a.partial_w[(size_t)b * nw + i];
    const int co = i / ncol, col = i - co * ncol;
    const int tap = col / a.cin, ci = col - tap * a.cin;
    a.grad_w[(co * a.cin + ci) * 9 + tap] = s;
  } else if (i < nw + a.cout) {
    const int co = i - nw;
    float s = 0.f;
    for (int b = 0; b < a.nblk; ++b) s += a.partial_b[(size_t)b * a.cout + co];
    a.grad_b[co] = s;
  }
}

// Sum of the loss partials in block order: loss = sum / norm.
__global__ void sg_loss_final_kernel(const double *partial, int nblk, double norm, double *loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[b];
  *loss = s / norm;
}

// ---------------------------------------------------------------------------
// Adam (Kingma and Ba 2015) on the float32 master weights, bias-corrected
// with the step count ts (>= 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sg_adam_kernel(const SgAdamArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const float g = a.grad[i];
  const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.w[i] -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
}

// ---------------------------------------------------------------------------
// Pack the float32 master weights into the bf16 operand layouts:
//   fwd1[cout][k]        k = tap*2 + cin (k < 18), zero beyond   (32 x 32)
//   fwd2/3[tap][cout][cin]                                       (9 x 32 x 32)
//   fwd4[tap][cin]                                               (9 x 32)
//   bwd2/3[tap][cin][cout]                                       (9 x 32 x 32)
//   bwd4[cin][k]         k = tap (k < 9), zero beyond            (32 x 32)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sg_pack_kernel(const SgPackArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const float *W1 = a.w + kSgOffW[0], *W2 = a.w + kSgOffW[1], *W3 = a.w + kSgOffW[2], *W4 = a.w + kSgOffW[3];
  if (i < 32 * 32) {                                   // fwd1 and bwd4
    const int co = i / 32, k = i % 32;
    a.fwd1[i] = k < 18 ? f2bf(W1[(co * 2 + (k & 1)) * 9 + (k >> 1)]) : (unsigned short)0;
    const int ci = co, tap = k;
    a.bwd4[i] = tap < 9 ? f2bf(W4[ci * 9 + tap]) : (unsigned short)0;
  }
  if (i < 9 * 32 * 32) {
    const int tap = i / 1024, rem = i % 1024, r0 = rem / 32, r1 = rem % 32;
    // forward: [tap][cout=r0][cin=r1]; backward: [tap][cin=r0][cout=r1]
    a.fwd2[i] = f2bf(W2[(r0 * 32 + r1) * 9 + tap]);
    a.fwd3[i] = f2bf(W3[(r0 * 32 + r1) * 9 + tap]);
    a.bwd2[i] = f2bf(W2[(r1 * 32 + r0) * 9 + tap]);
    a.bwd3[i] = f2bf(W3[(r1 * 32 + r0) * 9 + tap]);
  }
  if (i < 9 * 32) {
    const int tap = i / 32, ci = i % 32;
    a.fwd4[i] = f2bf(W4[ci * 9 + tap]);
  }
}

// ---------------------------------------------------------------------------
// Crop gather for training: sample c takes field f, rows y0.., cols x0..
// of the stored trajectories and writes T0, P and the normalised target
// (T16 - T0)/s as contiguous crop images.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sg_crop_kernel(const SgCropArgs a) {
  const long long n = (long long)a.ncrop * a.C * a.C;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i / ((long long)a.C * a.C));
  const int rem = (int)(i - (long long)c * a.C * a.C);
  const int y = rem / a.C, x = rem - y * a.C;
  const int f = a.crops[c * 3], y0 = a.crops[c * 3 + 1], x0 = a.crops[c * 3 + 2];
  const long long src = ((long long)f * a.Hf + y0 + y) * a.Wf + x0 + x;
  const float t0 = a.T0[src];
  a.T0c[i] = t0;
  a.Pc[i] = a.P[src];
  a.tgt[i] = (a.T16[src] - t0) / a.s;
}


// ---------------------------------------------------------------------------
// Residual check of one surrogate block (k steps from Tcur to Tnew).
//   r_mean: the mean of T obeys m' = m + cP*pbar + cz*(Tamb - m) exactly
//           (the clamped Laplacian sums to zero), so after k steps
//           m_k = A + (m_0 - A)(1 - cz)^k with A = Tamb + cP*pbar/cz;
//           r_mean = |mean(Tnew) - m_k| / max|Tnew|.
//   r_tile: on four 32x32 tiles the plain stencil is run k steps from Tcur
//           (with a k-cell halo, in LDS) and compared with Tnew:
//           r_tile = max |Tnew - plain| / max|Tnew|.
// r = max(r_mean, r_tile); the block's flag is r > threshold.
// The producer side writes per-block partials (sum Tcur, sum Tnew,
// max|Tnew|, all double) and the plain tile values; sg_check_final_kernel
// combines them in a fixed order.  Producers: the fused network kernel
// (partials of its own output tiles, plain tiles in blocks 0..3), or
// sg_check_partial_kernel after the per-layer network.
// ---------------------------------------------------------------------------
constexpr int kTile = 32, kHalo = 16, kRegion = kTile + 2 * kHalo;
constexpr int kNT = 512;            // threads of the check and fused kernels
constexpr int kNW = kNT / 64;

// Fixed-order sum / max over the block (result valid in thread 0).
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double *sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) r += sh[w];
  __syncthreads();
  return r;
}
template <int NW>
__device__ __forceinline__ float block_max_w(float v, float *sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) r = fmaxf(r, sh[w]);
  __syncthreads();
  return r;
}

// k plain steps over the (tile + k halo) region of check tile (y0, x0);
// writes the 32x32 tile values to out.  512 threads: thread (ty, tx) =
// (tid / 64, tid % 64) keeps rows 8*ty .. 8*ty+7 of region column tx in
// registers and publishes them in LDS (buf: 2 * kRegion^2 floats, double
// buffered) for its east / west neighbours and the strips above and below:
// one barrier per step.  Cells near a halo cut see a clamped neighbour that
// is not the true one; the error moves inward one cell per step and so
// never reaches the tile (the halo is k cells wide).
__device__ void check_plain_tile(const float *Tcur, const float *P, int ny, int nx, int ks, const HeatCoef &k,
                                 int y0, int x0, float *buf, float *out) {
  const int ry_lo = max(y0 - ks, 0), ry_hi = min(y0 + kTile + ks, ny);
  const int rx_lo = max(x0 - ks, 0), rx_hi = min(x0 + kTile + ks, nx);
  const int H = ry_hi - ry_lo, W = rx_hi - rx_lo;
  const int tx = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * 8;
  const bool col = tx < W;
  const int xw = tx > 0 ? tx - 1 : 0, xe = tx < W - 1 ? tx + 1 : W - 1;
  const int rn = r0 > 0 ? r0 - 1 : 0, rs = r0 + 8 < H ? r0 + 8 : H - 1;
  float v[8], pw[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int yy = min(r0 + i, H - 1);
    const long long g = (long long)(ry_lo + yy) * nx + rx_lo + (col ? tx : 0);
    v[i] = Tcur[g];
    pw[i] = P[g];
  }
  float *A = buf, *B = buf + kRegion * kRegion;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (col && r0 + i < H) A[(r0 + i) * kRegion + tx] = v[i];
  __syncthreads();
  for (int s = 0; s < ks; ++s) {
    float w[8], e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int yy = min(r0 + i, H - 1);
      w[i] = A[yy * kRegion + xw];
      e[i] = A[yy * kRegion + xe];
    }
    const float top = A[rn * kRegion + tx], bot = A[rs * kRegion + tx];
    float nv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int yy = r0 + i;
      const float n = yy == 0 ? v[i] : (i == 0 ? top : v[i - 1]);
      const float so = yy >= H - 1 ? v[i] : (i == 7 ? bot : v[i + 1]);
      nv[i] = heat_update(v[i], n, so, w[i], e[i], pw[i], k);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      v[i] = nv[i];
      if (col && r0 + i < H) B[(r0 + i) * kRegion + tx] = v[i];
    }
    __syncthreads();
    float *t = A; A = B; B = t;
  }
  for (int c = threadIdx.x; c < kTile * kTile; c += kNT) {
    const int yy = c >> 5, xx = c & 31;
    out[c] = A[(y0 + yy - ry_lo) * kRegion + (x0 + xx - rx_lo)];
  }
}

// Final pass: one block of 1024 threads combines the per-block partials in a
// fixed order (thread i takes partials i, i+1024, ..., then a fixed tree
// over the waves), compares the tiles, sets the flag and logs r.
__global__ __launch_bounds__(1024) void sg_check_final_kernel(const SgCheckArgs a) {
  __shared__ double dsh[2][16];
  __shared__ float fsh[2][16];
  double sc = 0.0, sn = 0.0;
  float mx = 0.f, dt = 0.f;
  for (int b = threadIdx.x; b < a.nred; b += 1024) {
    sc += a.partial[b * 3 + 0];
    sn += a.partial[b * 3 + 1];
    mx = fmaxf(mx, (float)a.partial[b * 3 + 2]);
  }
  for (int q = threadIdx.x; q < 4 * kTile * kTile; q += 1024) {
    const int t = q >> 10, yy = (q >> 5) & 31, xx = q & 31;
    const float v = a.Tnew[(long long)(a.tile_y[t] + yy) * a.nx + a.tile_x[t] + xx];
    dt = fmaxf(dt, fabsf(v - a.plain[q]));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sc += __shfl_xor(sc, o, 64);
    sn += __shfl_xor(sn, o, 64);
    mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    dt = fmaxf(dt, __shfl_xor(dt, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    dsh[0][w] = sc; dsh[1][w] = sn;
    fsh[0][w] = mx; fsh[1][w] = dt;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double S1 = 0.0, S2 = 0.0;
  float MX = 0.f, DT = 0.f;
  for (int i = 0; i < 16; ++i) {
    S1 += dsh[0][i]; S2 += dsh[1][i];
    MX = fmaxf(MX, fsh[0][i]); DT = fmaxf(DT, fsh[1][i]);
  }
  const SgCheckTail &c = a.tail;
  const double n = (double)a.ny * a.nx;
  const double cP = a.k.cP, cz = a.k.cz, Tamb = a.k.Tamb;
  const double A = Tamb + cP * (*c.psum / n) / cz;
  const double mk = A + (S1 / n - A) * c.decay;
  const double scale = MX > 0.f ? (double)MX : 1.0;
  const double r = fmax(fabs(S2 / n - mk) / scale, (double)DT / scale);
  const int f = r > c.threshold ? 1 : 0;
  *c.flag = f;
  const long long cnt = c.counters[0];
  if (cnt >= 0 && cnt < c.hist_cap) c.hist[cnt] = r;
  c.counters[0] = cnt + 1;
  c.counters[1] += f;
}

// Producer after the per-layer network: blocks < nred reduce fixed chunks
// of the field, blocks nred..nred+3 run the plain check tiles.
__global__ __launch_bounds__(kNT) void sg_check_partial_kernel(const SgCheckArgs a) {
  __shared__ double dsh[kNW];
  __shared__ float fsh[kNW];
  __shared__ float buf[2 * kRegion * kRegion];
  const long long n = (long long)a.ny * a.nx;
  if ((int)blockIdx.x >= a.nred) {
    const int t = blockIdx.x - a.nred;
    check_plain_tile(a.Tcur, a.P, a.ny, a.nx, a.ksteps, a.k, a.tile_y[t], a.tile_x[t], buf,
                     a.plain + t * kTile * kTile);
  } else {
    const long long lo = n * blockIdx.x / a.nred, hi = n * (blockIdx.x + 1) / a.nred;
    double sc = 0.0, sn = 0.0;
    float mx = 0.f;
    for (long long i = lo + threadIdx.x; i < hi; i += kNT) {
      sc += (double)a.Tcur[i];
      const float v = a.Tnew[i];
      sn += (double)v;
      mx = fmaxf(mx, fabsf(v));
    }
    const double s1 = block_sum_w<kNW>(sc, dsh);
    const double s2 = block_sum_w<kNW>(sn, dsh);
    const float m = block_max_w<kNW>(mx, fsh);
    if (threadIdx.x == 0) {
      a.partial[blockIdx.x * 3 + 0] = s1;
      a.partial[blockIdx.x * 3 + 1] = s2;
      a.partial[blockIdx.x * 3 + 2] = (double)m;
    }
  }
}

void sg_make_check(Launch &L0, Launch &L1, const SgCheckArgs &a) {
  L0.set((const void *)sg_check_partial_kernel, dim3(a.nred + 4), dim3(kNT), 0, a);
  L1.set((const void *)sg_check_final_kernel, dim3(1), dim3(1024), 0, a);
}

void sg_make_check_final(Launch &L, const SgCheckArgs &a) {
  L.set((const void *)sg_check_final_kernel, dim3(1), dim3(1024), 0, a);
}

int sg_check_tile() { return kTile; }

// ---------------------------------------------------------------------------
// Fused inference: one block evaluates the whole network on a 16x32 output
// tile with every activation held in LDS, so HBM traffic is T0 and P in and
// T_k out.  Each layer is computed on the tile grown by the receptive field
// still ahead of it:
//   input (t, p)   24 x 40   bf16 pairs
//   layer 1 out    22 x 38   32 ch   (buffer A)
//   layer 2 out    20 x 36   32 ch   (buffer B)
//   layer 3 out    18 x 34   32 ch   (buffer A)
//   layer 4        16 x 32
// A region pixel takes its image coordinates clamped into the field and
// reads taps at clamped coordinates, which is replicate padding at every
// layer (a clamped tap always lies inside the previous, larger region).
// Layers 1-3 are the forward implicit GEMM of sg_conv_fwd_kernel with the
// B fragments read from LDS.  The weight fragments of layers 2 and 3 are
// kept in LDS in fragment order (a wave's load of one fragment is 1 KiB of
// consecutive bytes) and a wave takes the current layer's 18 fragments into
// registers when the layer starts, which leaves room for three waves per
// SIMD (12 per block).  Layer 4 (one output channel) is done in transposed
// form: one MFMA per 16 pixels of layer 3 gives every pixel's contribution
// to each of the 9 taps, D[pixel][tap], and an output pixel sums the 9
// entries of its clamped neighbours.
// Activations are pixel-major, 64 bytes per pixel; the 16-byte channel
// chunk c of pixel p sits in slot (c + (p >> 1)) & 3, so that the eight
// consecutive pixels of a 128-byte load pass use eight distinct slots.
// Blocks 0..3 run the plain check tiles; blocks 4.. are persistent over the
// output tiles (tile i goes to block 4 + i % nnet) and write the check
// partials of the tiles they produced.
// ---------------------------------------------------------------------------
namespace fz {
constexpr int TH = 16, TW = 32;
constexpr int H0 = TH + 8, W0 = TW + 8, N0 = H0 * W0;
constexpr int H1 = TH + 6, W1 = TW + 6, N1 = H1 * W1;
constexpr int H2 = TH + 4, W2 = TW + 4, N2 = H2 * W2;
constexpr int H3 = TH + 2, W3 = TW + 2, N3 = H3 * W3;
constexpr int G1 = (N1 + 15) / 16, G2 = (N2 + 15) / 16, G3 = (N3 + 15) / 16;
constexpr int kPix = 64;                              // bytes per pixel (32 bf16 channels)
constexpr int kW = 12;                                // waves per block
constexpr int kT = 64 * kW;                           // threads per block
constexpr int kIn = 0;                                // N0 uint
constexpr int kA = kIn + N0 * 4;                      // N1 * kPix bytes
constexpr int kB = kA + N1 * kPix;                    // N2 * kPix bytes
constexpr int kWt = kB + N2 * kPix;                   // weight fragments, 16 bytes per lane:
constexpr int kWf2 = 0, kWf3 = 9 * 2 * 64, kWf1 = 2 * 9 * 2 * 64, kWf4 = kWf1 + 2 * 64;   //  layers 2, 3 [tap][m][lane]; 1 [m][lane]; 4 [lane]
constexpr int kNWf = kWf4 + 64;
constexpr int kBytes = kWt + kNWf * 16;
static_assert(N3 * 9 * 4 <= N2 * kPix, "layer-4 partials must fit buffer B");
static_assert(2 * kRegion * kRegion * 4 <= kWt, "check tile must fit");
static_assert(kA % 16 == 0 && kB % 16 == 0 && kWt % 16 == 0, "16-byte aligned buffers");
static_assert(N0 <= 2 * kT, "two input pixels per thread");
static_assert(TH * TW <= kT, "one output pixel per thread");
// byte offset of the 16-byte channel chunk c of pixel p
__device__ __forceinline__ int chunk(int p, int c) { return p * kPix + (((c + (p >> 1)) & 3) << 4); }
}  // namespace fz

// Source pixel (in the previous region) of tap (dy, dx) for region pixel p.
// Interior tiles (EDGE = false): no clamping, so the nine taps are the
// pixel's base index plus compile-time offsets.  Edge tiles clamp each
// coordinate into the field.
template <int Wr, bool EDGE>
struct TapSrc {
  int base;                 // interior: index of tap (0, 0)
  int ro[3], co[3];         // edge: row and column offsets per dy / dx
  __device__ __forceinline__ TapSrc(int p, int oy, int ox, int H, int W) {
    const int i = p / Wr, j = p - (p / Wr) * Wr;
    if constexpr (!EDGE) {
      base = p + 2 * i;
    } else {
      const int cy = clampi(oy + i, H), cx = clampi(ox + j, W);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ro[d] = (clampi(cy + d - 1, H) - oy + 1) * (Wr + 2);
        co[d] = clampi(cx + d - 1, W) - ox + 1;
      }
    }
  }
  __device__ __forceinline__ int operator()(int tap) const {
    if constexpr (!EDGE) return base + (tap / 3) * (Wr + 2) + tap % 3;
    else return ro[tap / 3] + co[tap % 3];
  }
};

// Epilogue of a 32-channel layer (bias already in the accumulator): GELU,
// bf16, into the region buffer.  Lane (r, kq) holds channels m*16 + kq*4 ..
// +3 of pixel p.
__device__ __forceinline__ void store_act(unsigned char *dst, int p, int kq, const f32x4 (&acc)[2]) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    uint2 packed;
    packed.x = f2bf2(gelu(acc[m][0]), gelu(acc[m][1]));
    packed.y = f2bf2(gelu(acc[m][2]), gelu(acc[m][3]));
    // channels m*16 + kq*4 .. +3: chunk 2m + kq/2, bytes (kq & 1) * 8
    *reinterpret_cast<uint2 *>(dst + fz::chunk(p, 2 * m + (kq >> 1)) + (kq & 1) * 8) = packed;
    __builtin_amdgcn_sched_barrier(0);   // four activations at a time (registers)
  }
}

__device__ __forceinline__ void bias_init(f32x4 (&acc)[2], const float *bias, int kq) {
  acc[0] = *reinterpret_cast<const f32x4 *>(bias + kq * 4);
  acc[1] = *reinterpret_cast<const f32x4 *>(bias + 16 + kq * 4);
}

// One 32 -> 32 layer over a region (Wr wide, N pixels, G groups of 16);
// wf: the layer's weight fragments in LDS, [tap][m][lane].
template <int Wr, int N, int G, bool EDGE>
__device__ __forceinline__ void fused_layer32(const unsigned char *src, unsigned char *dst, const bf16x8 *wf,
                                              const float *bias, int oy, int ox, int H, int W) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  bf16x8 wa[9][2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int m = 0; m < 2; ++m) wa[tap][m] = wf[(tap * 2 + m) * 64 + lane];
  for (int g = wave; g < G; g += fz::kW) {
    const int p = min(g * 16 + r, N - 1);
    const TapSrc<Wr, EDGE> ts(p, oy, ox, H, W);
    f32x4 acc[2];
    bias_init(acc, bias, kq);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const bf16x8 B = ld_frag(reinterpret_cast<const unsigned short *>(src + fz::chunk(ts(tap), kq)));
      acc[0] = mfma(wa[tap][0], B, acc[0]);
      acc[1] = mfma(wa[tap][1], B, acc[1]);
      // at most three taps' operands in flight (register room for three
      // waves per SIMD)
      if (tap % 3 == 2) __builtin_amdgcn_sched_barrier(0);
    }
    const int po = g * 16 + r;
    if (po < N) store_act(dst, po, kq, acc);
  }
}

// The network on one 16x32 output tile; in0 holds the tile's input region.
// Returns after the last barrier that orders this tile's LDS use; the
// output phase follows in the caller.
template <bool EDGE>
__device__ __forceinline__ void fused_tile(const SgFusedArgs &a, unsigned char *sm, const float *sbias, int y0,
                                           int x0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const unsigned *in0 = reinterpret_cast<const unsigned *>(sm + fz::kIn);
  unsigned char *bA = sm + fz::kA, *bB = sm + fz::kB;
  const bf16x8 *wf = reinterpret_cast<const bf16x8 *>(sm + fz::kWt);
  float *Dl = reinterpret_cast<float *>(bB);
  // layer 1 (2 -> 32): k = tap*2 + cin; lane kq gathers taps kq*4 .. kq*4+3
  for (int g = wave; g < fz::G1; g += fz::kW) {
    const int p = min(g * 16 + r, fz::N1 - 1);
    const TapSrc<fz::W1, EDGE> ts(p, y0 - 3, x0 - 3, a.H, a.W);
    unsigned u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int tap = kq * 4 + i;
      u[i] = tap < 9 ? in0[ts(tap < 9 ? tap : 0)] : 0u;
    }
    const bf16x8 B = __builtin_bit_cast(bf16x8, uint4{u[0], u[1], u[2], u[3]});
    f32x4 acc[2];
    bias_init(acc, sbias, kq);
    acc[0] = mfma(wf[fz::kWf1 + lane], B, acc[0]);
    acc[1] = mfma(wf[fz::kWf1 + 64 + lane], B, acc[1]);
    const int po = g * 16 + r;
    if (po < fz::N1) store_act(bA, po, kq, acc);
  }
  __syncthreads();
  fused_layer32<fz::W2, fz::N2, fz::G2, EDGE>(bA, bB, wf + fz::kWf2, sbias + 32, y0 - 2, x0 - 2, a.H, a.W);
  __syncthreads();
  fused_layer32<fz::W3, fz::N3, fz::G3, EDGE>(bB, bA, wf + fz::kWf3, sbias + 64, y0 - 1, x0 - 1, a.H, a.W);
  __syncthreads();
  // layer 4, transposed: D[pixel][tap] = sum_cin act3[pixel][cin] W4[tap][cin]
  for (int g = wave; g < fz::G3; g += fz::kW) {
    const int p = min(g * 16 + r, fz::N3 - 1);
    const bf16x8 A = ld_frag(reinterpret_cast<const unsigned short *>(bA + fz::chunk(p, kq)));
    const f32x4 d = mfma(A, wf[fz::kWf4 + lane], f32x4{0.f, 0.f, 0.f, 0.f});
    if (r < 9) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int pp = g * 16 + kq * 4 + j;
        if (pp < fz::N3) Dl[pp * 9 + r] = d[j];
      }
    }
  }
  __syncthreads();
}

// Output pixel (i, j) of the tile: y = b4 + the nine tap partials at the
// (clamped) neighbours.
template <bool EDGE>
__device__ __forceinline__ float fused_out(const SgFusedArgs &a, const float *Dl, int y0, int x0, int i, int j) {
  float acc = 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    int q;
    if constexpr (!EDGE) {
      q = (i + tap / 3) * fz::W3 + j + tap % 3;
    } else {
      const int sy = clampi(y0 + i + tap / 3 - 1, a.H) - (y0 - 1);
      const int sx = clampi(x0 + j + tap % 3 - 1, a.W) - (x0 - 1);
      q = sy * fz::W3 + sx;
    }
    acc += Dl[q * 9 + tap];
  }
  return acc;
}

__global__ __launch_bounds__(fz::kT) void sg_fused_kernel(const SgFusedArgs a) {
  __shared__ __align__(16) unsigned char sm[fz::kBytes];
  __shared__ __align__(16) float sbias[100];
  __shared__ float t0s[2][fz::TH * fz::TW];   // by tile parity: written before the
                                              // previous tile's output is read out
  __shared__ double dsh[fz::kW];
  __shared__ float fsh[fz::kW];
  if (blockIdx.x < 4) {
    const int t = blockIdx.x;
    check_plain_tile(a.T0, a.P, a.H, a.W, a.ksteps, a.k, a.tile_y[t], a.tile_x[t], reinterpret_cast<float *>(sm),
                     a.plain + t * kTile * kTile);
    return;
  }
  const int nb = blockIdx.x - 4;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kq = lane >> 4;
  unsigned *in0 = reinterpret_cast<unsigned *>(sm + fz::kIn);
  const float *Dl = reinterpret_cast<const float *>(sm + fz::kB);
  if (threadIdx.x < 96) sbias[threadIdx.x] = a.bias[kSgOffB[threadIdx.x >> 5] + (threadIdx.x & 31)];
  if (threadIdx.x == 96) sbias[96] = a.bias[kSgOffB[3]];

  // weight fragments in LDS in fragment order (one wave's fragment = 1 KiB
  // of consecutive bytes): layers 2, 3 [tap][m][lane] (A operands), layer 1
  // [m][lane] (A), layer 4 [lane] (the B operand of the transposed layer)
  {
    bf16x8 *wf = reinterpret_cast<bf16x8 *>(sm + fz::kWt);
    for (int e = threadIdx.x; e < fz::kNWf; e += fz::kT) {
      const int ln = e % 64, rr = ln & 15, qq = ln >> 4;
      bf16x8 v;
      if (e < fz::kWf1) {
        const int l = e / fz::kWf3, tap = (e / (2 * 64)) % 9, m = (e / 64) % 2;
        v = ld_frag((l == 0 ? a.w2 : a.w3) + (tap * 32 + m * 16 + rr) * 32 + qq * 8);
      } else if (e < fz::kWf4) {
        const int m = (e - fz::kWf1) / 64;
        v = ld_frag(a.w1 + (m * 16 + rr) * 32 + qq * 8);
      } else {
        v = rr < 9 ? ld_frag(a.w4 + rr * 32 + qq * 8) : __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
      }
      wf[e] = v;
    }
  }

  // input values of the 24 x 40 region, two per thread, loaded one tile ahead
  float pT[2], pP[2];
  auto fetch = [&](int tile) {
    const int y0 = (tile / a.tiles_x) * fz::TH, x0 = (tile % a.tiles_x) * fz::TW;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = min((int)threadIdx.x + q * fz::kT, fz::N0 - 1);
      const int i = p / fz::W0, j = p - (p / fz::W0) * fz::W0;
      const long long g = (long long)clampi(y0 - 4 + i, a.H) * a.W + clampi(x0 - 4 + j, a.W);
      pT[q] = a.T0[g];
      pP[q] = a.P[g];
    }
  };
  if (nb < a.ntiles) fetch(nb);

  double s_cur = 0.0, s_new = 0.0;
  float mx = 0.f;
  int par = 0;
  for (int tile = nb; tile < a.ntiles; tile += a.nnet, par ^= 1) {
    const int y0 = (tile / a.tiles_x) * fz::TH, x0 = (tile % a.tiles_x) * fz::TW;
    // network input; the tile's own T0 values are kept for the output
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = threadIdx.x + q * fz::kT;
      if (p < fz::N0) {
        const float t = (pT[q] - 333.0f) / 10.0f;
        const float u = (pP[q] - 0.5f) / 0.29f;
        in0[p] = f2bf2(t, u);
        const int i = p / fz::W0 - 4, j = p - (p / fz::W0) * fz::W0 - 4;
        if (i >= 0 && i < fz::TH && j >= 0 && j < fz::TW) t0s[par][i * fz::TW + j] = pT[q];
      }
    }
    __syncthreads();
    if (tile + a.nnet < a.ntiles) fetch(tile + a.nnet);
    const bool interior = y0 >= 4 && x0 >= 4 && y0 + fz::TH + 4 <= a.H && x0 + fz::TW + 4 <= a.W;
    if (interior) fused_tile<false>(a, sm, sbias, y0, x0);
    else fused_tile<true>(a, sm, sbias, y0, x0);
    // output (one pixel per thread)
    const int i = threadIdx.x >> 5, j = threadIdx.x & 31;
    const int yy = y0 + i, xx = x0 + j;
    if (i < fz::TH && yy < a.H && xx < a.W) {
      const float acc = interior ? fused_out<false>(a, Dl, y0, x0, i, j) : fused_out<true>(a, Dl, y0, x0, i, j);
      const float y = acc + sbias[96];
      const float t0 = t0s[par][i * fz::TW + j];
      const float tn = t0 + a.s * y;
      a.Tout[(long long)yy * a.W + xx] = tn;
      s_cur += (double)t0;
      s_new += (double)tn;
      mx = fmaxf(mx, fabsf(tn));
    }
    // buffer B (D) is next written after two more barriers, t0s[par] after
    // three; in0 and buffer A are no longer read by this tile.
  }
  const double s1 = block_sum_w<fz::kW>(s_cur, dsh);
  const double s2 = block_sum_w<fz::kW>(s_new, dsh);
  const float m = block_max_w<fz::kW>(mx, fsh);
  if (threadIdx.x == 0) {
    a.partial[nb * 3 + 0] = s1;
    a.partial[nb * 3 + 1] = s2;
    a.partial[nb * 3 + 2] = (double)m;
  }
}

void sg_make_fused(Launch &L, const SgFusedArgs &a) {
  L.set((const void *)sg_fused_kernel, dim3(a.nnet + 4), dim3(fz::kT), 0, a);
}

int sg_fused_tiles(int H, int W, int *tiles_x) {
  *tiles_x = (W + fz::TW - 1) / fz::TW;
  return ((H + fz::TH - 1) / fz::TH) * *tiles_x;
}

// ---------------------------------------------------------------------------
// Launch helpers (host).
// ---------------------------------------------------------------------------
static unsigned nblk_pix(long long npix, int per) { return (unsigned)((npix + per - 1) / per); }

hipError_t sg_launch_input(const SgInputArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sg_input_kernel, dim3(nblk_pix(a.npix, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

void sg_make_conv(Launch &L, const SgConvArgs &a, int layer) {
  const dim3 g(nblk_pix(a.npix, 256)), b(256);
  switch (layer) {
    case 0: L.set((const void *)sg_conv_fwd_kernel<2, 32>, g, b, 0, a); break;
    case 1:
    case 2: L.set((const void *)sg_conv_fwd_kernel<32, 32>, g, b, 0, a); break;
    default: L.set((const void *)sg_conv_fwd_kernel<32, 1>, g, b, 0, a); break;
  }
}

void sg_make_input(Launch &L, const SgInputArgs &a) {
  L.set((const void *)sg_input_kernel, dim3(nblk_pix(a.npix, 256)), dim3(256), 0, a);
}

hipError_t sg_launch_loss(const SgLossArgs &a, int nblk, double norm, double *loss, hipStream_t s) {
  hipLaunchKernelGGL(sg_loss_kernel, dim3(nblk), dim3(256), 0, s, a);
  hipLaunchKernelGGL(sg_loss_final_kernel, dim3(1), dim3(64), 0, s, (const double *)a.partial, nblk, norm, loss);
  return hipGetLastError();
}

hipError_t sg_launch_dgrad(const SgDgradArgs &a, int cout, hipStream_t s) {
  const dim3 g(nblk_pix(a.npix, 256)), b(256);
  if (cout == 32) hipLaunchKernelGGL(sg_dgrad_kernel<32>, g, b, 0, s, a);
  else hipLaunchKernelGGL(sg_dgrad_kernel<1>, g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t sg_launch_wgrad(const SgWgradArgs &a, int cin, int cout, int nblk, hipStream_t s) {
  const dim3 g(nblk), b(256);
  if (cin == 2) hipLaunchKernelGGL((sg_wgrad_kernel<2, 32>), g, b, 0, s, a);
  else if (cout == 32) hipLaunchKernelGGL((sg_wgrad_kernel<32, 32>), g, b, 0, s, a);
  else hipLaunchKernelGGL((sg_wgrad_kernel<32, 1>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t sg_launch_reduce(const SgReduceArgs &a, hipStream_t s) {
  const int n = a.cout * 9 * a.cin + a.cout;
  hipLaunchKernelGGL(sg_grad_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t sg_launch_adam(const SgAdamArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sg_adam_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t sg_launch_pack(const SgPackArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sg_pack_kernel, dim3((9 * 32 * 32 + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t sg_launch_crop(const SgCropArgs &a, hipStream_t s) {
  const long long n = (long long)a.ncrop * a.C * a.C;
  hipLaunchKernelGGL(sg_crop_kernel, dim3(nblk_pix(n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace kb
