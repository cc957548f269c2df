// Internal declarations of the surrogate kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kb_internal.h"

namespace kb {

// Weight vector layout (float32, canonical order):
//   W1[32][2][3][3], b1[32], W2[32][32][3][3], b2[32],
//   W3[32][32][3][3], b3[32], W4[1][32][3][3], b4[1]
constexpr int kSgNW = 19393;
constexpr int kSgOffW[4] = {0, 608, 9856, 19104};
constexpr int kSgOffB[4] = {576, 9824, 19072, 19392};
constexpr int kSgCin[4] = {2, 32, 32, 32};
constexpr int kSgCout[4] = {32, 32, 32, 1};
constexpr int kSgWgradBlocks = 256;        // partial sums per weight gradient

struct SgInputArgs {
  const float *T0, *P;
  unsigned short *x;        // [npix][2] bf16
  long long npix;
};

struct SgConvArgs {
  const unsigned short *in; // [npix][cin] bf16
  const unsigned short *w;  // packed forward weights of the layer
  const float *bias;
  float *z;                 // [npix][32] pre-activations (optional)
  unsigned short *out;      // [npix][32] bf16 activations (hidden layers)
  float *y;                 // [npix] network output (last layer, optional)
  const float *T0;          // last layer: Tout = T0 + s*y (optional)
  float *Tout;
  float s;
  long long npix;
  int H, W;
};

struct SgLossArgs {
  const float *y, *target;
  float *g;                 // [npix] dL/dy
  double *partial;          // [nblk]
  float norm;
  long long npix;
};

struct SgDgradArgs {
  const float *g;           // [npix][cout] gradient of the layer's output
  const unsigned short *w;  // packed backward weights of the layer
  const float *z;           // [npix][32] pre-activations of the layer's input
  float *gout;              // [npix][32] gradient of those pre-activations
  long long npix;
  int H, W;
};

struct SgWgradArgs {
  const float *g;           // [npix][cout]
  const unsigned short *x;  // [npix][cin] bf16 layer input
  float *partial_w;         // [nblk][cout][9*cin]
  float *partial_b;         // [nblk][cout]
  int nimg, H, W;
};

struct SgReduceArgs {
  const float *partial_w, *partial_b;
  float *grad_w, *grad_b;   // canonical positions in the gradient vector
  int nblk, cin, cout;
};

struct SgAdamArgs {
  float *w, *m, *v;
  const float *grad;
  float lr, b1, b2, eps, c1, c2;
  int n;
};

struct SgPackArgs {
  const float *w;
  unsigned short *fwd1, *fwd2, *fwd3, *fwd4, *bwd2, *bwd3, *bwd4;
};

struct SgCropArgs {
  const float *T0, *P, *T16;   // [nfield][Hf][Wf]
  const int *crops;            // [ncrop][3]: field, y0, x0
  float *T0c, *Pc, *tgt;       // [ncrop][C][C]
  int ncrop, C, Hf, Wf;
  float s;
};

hipError_t sg_launch_input(const SgInputArgs &a, hipStream_t s);
hipError_t sg_launch_loss(const SgLossArgs &a, int nblk, double norm, double *loss, hipStream_t s);
hipError_t sg_launch_dgrad(const SgDgradArgs &a, int cout, hipStream_t s);
hipError_t sg_launch_wgrad(const SgWgradArgs &a, int cin, int cout, int nblk, hipStream_t s);
hipError_t sg_launch_reduce(const SgReduceArgs &a, hipStream_t s);
hipError_t sg_launch_adam(const SgAdamArgs &a, hipStream_t s);
hipError_t sg_launch_pack(const SgPackArgs &a, hipStream_t s);
hipError_t sg_launch_crop(const SgCropArgs &a, hipStream_t s);

}  // namespace kb

namespace kb {

// Inputs and outputs of the residual check's final pass.
struct SgCheckTail {
  const double *psum;             // sum of P over the field
  double decay;                   // (1 - c/Rz)^k of the mean recurrence (host pow)
  double threshold;
  int *flag;                      // set to (r > threshold)
  double *hist;                   // r of every checked block
  long long hist_cap;
  long long *counters;            // [0] blocks checked, [1] fallbacks
};

struct SgCheckArgs {
  const float *Tcur, *Tnew, *P;   // [ny][nx]
  int ny, nx, ksteps;
  HeatCoef k;                      // coefficients of the plain step
  int tile_y[4], tile_x[4];       // 32x32 check tiles
  double *partial;                // [nred][3]: sum Tcur, sum Tnew, max|Tnew|
  int nred;
  float *plain;                   // [4][32*32] plain k-step values of the tiles
  SgCheckTail tail;
};

// Fused inference of the whole network plus the residual check's
// producer side (per-block partials, plain tiles).
struct SgFusedArgs {
  const float *T0, *P;
  float *Tout;
  const unsigned short *w1, *w2, *w3, *w4;   // packed forward weights
  const float *bias;                          // float32 weight vector (biases at kSgOffB)
  double *partial;                            // [nnet][3]
  float *plain;                               // [4][32*32]
  HeatCoef k;
  float s;
  int H, W, tiles_x, ntiles, nnet, ksteps;
  int tile_y[4], tile_x[4];
};

void sg_make_conv(Launch &L, const SgConvArgs &a, int layer);
void sg_make_input(Launch &L, const SgInputArgs &a);
void sg_make_check(Launch &L0, Launch &L1, const SgCheckArgs &a);
void sg_make_check_final(Launch &L, const SgCheckArgs &a);
void sg_make_fused(Launch &L, const SgFusedArgs &a);
int sg_fused_tiles(int H, int W, int *tiles_x);   // output tiles of the fused kernel
int sg_check_tile();
}  // namespace kb
