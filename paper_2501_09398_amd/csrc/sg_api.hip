// C ABI of the learned k-step surrogate: problem set-up, the k-step block
// that a graph batches (network, residual check, predicated fallback), and
// the training entry points (loss and gradient, Adam step).
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <new>

#include "kb_internal.h"
#include "sg_internal.h"

using namespace kb;

namespace kb {

constexpr int kSgHistCap = 4096;
constexpr int kSgRedBlocks = 256;
constexpr int kSgLossBlocks = 256;
constexpr int kSgMaxCrops = 1024;
constexpr int kSgMaxNet = 1024;           // persistent blocks of the fused kernel

// Workspace offsets of the surrogate problem.
struct SgLayout {
  size_t total = 0;
  size_t T[2], P, x, act[2];
  size_t T0c, Pc, tgt, xt, a[3], z[3], yt, g4, g[3], pw, pb, lossp, loss, crops;
  size_t w, grad, m, v, fwd1, fwd2, fwd3, fwd4, bwd2, bwd3, bwd4;
  size_t chk, plain, psum, flag, hist, counters;
};

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

bool sg_layout(const int64_t *shape, int ndim, SgLayout &L) {
  if (!shape || (ndim != 2 && ndim != 3)) return false;
  const int64_t ny = shape[0], nx = shape[1], m = ndim == 3 ? shape[2] : 0;
  if (ny < 32 || nx < 32 || ny > 16384 || nx > 16384 || m < 0 || m > ((int64_t)1 << 24)) return false;
  const size_t n = (size_t)(ny * nx);
  size_t o = 0;
  auto add = [&](size_t bytes) { size_t r = o; o = al(o + (bytes ? bytes : 4)); return r; };
  L.T[0] = add(n * 4); L.T[1] = add(n * 4); L.P = add(n * 4);
  L.x = add(n * 4); L.act[0] = add(n * 64); L.act[1] = add(n * 64);
  const size_t mm = (size_t)m;
  L.T0c = add(mm * 4); L.Pc = add(mm * 4); L.tgt = add(mm * 4); L.xt = add(mm * 4);
  for (int l = 0; l < 3; ++l) { L.a[l] = add(mm * 64); L.z[l] = add(mm * 128); }
  L.yt = add(mm * 4); L.g4 = add(mm * 4);
  for (int l = 0; l < 3; ++l) L.g[l] = add(mm * 128);
  L.pw = add((size_t)kSgWgradBlocks * 32 * 288 * 4); L.pb = add((size_t)kSgWgradBlocks * 32 * 4);
  L.lossp = add(kSgLossBlocks * 8); L.loss = add(8); L.crops = add(kSgMaxCrops * 3 * 4);
  L.w = add(kSgNW * 4); L.grad = add(kSgNW * 4); L.m = add(kSgNW * 4); L.v = add(kSgNW * 4);
  L.fwd1 = add(1024 * 2); L.fwd2 = add(9216 * 2); L.fwd3 = add(9216 * 2); L.fwd4 = add(288 * 2);
  L.bwd2 = add(9216 * 2); L.bwd3 = add(9216 * 2); L.bwd4 = add(1024 * 2);
  L.chk = add((size_t)(kSgMaxNet > kSgRedBlocks ? kSgMaxNet : kSgRedBlocks) * 3 * 8);
  L.plain = add(4 * 32 * 32 * 4); L.psum = add(8); L.flag = add(4);
  L.hist = add(kSgHistCap * 8); L.counters = add(16);
  L.total = o;
  return true;
}

struct SgState {
  SgLayout L;
  unsigned char *ws = nullptr;
  long long n = 0, train_pix = 0;
  int ksteps = 16;
  float s = 0.8f;
  double threshold = 1e-3;
  long long adam_t = 0;
  long long last_m = 0;                    // pixels of the last training batch (tape fields)
  int tile_y[4], tile_x[4];
  int tiles_x = 0, ntiles = 0, nnet = 0;   // fused kernel: output tiles, persistent blocks
  template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

size_t sg_workspace_bytes(const int64_t *shape, int ndim) {
  SgLayout L;
  return sg_layout(shape, ndim, L) ? L.total : 0;
}

static SgPackArgs pack_args(const SgState &S) {
  return SgPackArgs{S.at<float>(S.L.w), S.at<unsigned short>(S.L.fwd1), S.at<unsigned short>(S.L.fwd2),
                    S.at<unsigned short>(S.L.fwd3), S.at<unsigned short>(S.L.fwd4),
                    S.at<unsigned short>(S.L.bwd2), S.at<unsigned short>(S.L.bwd3),
                    S.at<unsigned short>(S.L.bwd4)};
}

hipError_t sg_repack(kb_problem *h) { return sg_launch_pack(pack_args(*h->sg), h->stream); }

// P changed: recompute its sum (the residual check's mean term needs it).
hipError_t sg_power_changed(kb_problem *h) {
  SgState &S = *h->sg;
  return reduce_sum(h->P, S.n, h->partials, S.at<double>(S.L.psum), h->stream);
}

int sg_create(kb_problem *h, const int64_t *shape, int ndim, const double *c, int nc, uint64_t seed,
              std::string &err) {
  SgState *S = new (std::nothrow) SgState();
  if (!S) { err = "host allocation failed"; return KB_ENOMEM; }
  h->sg = S;
  sg_layout(shape, ndim, S->L);
  S->ws = h->ws;
  S->n = shape[0] * shape[1];
  S->train_pix = ndim == 3 ? shape[2] : 0;
  if (nc == 8) {
    S->s = (float)c[5];
    S->threshold = c[6];
    S->ksteps = (int)c[7];
    if (!(S->s > 0) || !(c[6] >= 0) || (double)S->ksteps != c[7] || S->ksteps < 1 ||
        S->ksteps > heat2d_tile_max_depth()) {
      err = "surrogate coefficients: s > 0, threshold >= 0, 1 <= k <= 16";
      return KB_EINVAL;
    }
  }
  h->ny = shape[0];
  h->nx = shape[1];
  h->nz = 1;
  h->Tbuf[0] = S->at<float>(S->L.T[0]);
  h->Tbuf[1] = S->at<float>(S->L.T[1]);
  h->P = S->at<float>(S->L.P);
  h->K = 3;
  // fused kernel: one persistent block per compute unit (at most one tile each)
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu < 1) {
    err = "hipDeviceGetAttribute failed";
    return KB_EHIP;
  }
  S->ntiles = sg_fused_tiles((int)shape[0], (int)shape[1], &S->tiles_x);
  S->nnet = std::min(std::min(S->ntiles, ncu), kSgMaxNet);
  // check tiles: four 32x32 tiles at seeded positions
  for (int t = 0; t < 4; ++t) {
    S->tile_y[t] = (int)host_randint(seed, 10, 2 * t, h->ny - 31);
    S->tile_x[t] = (int)host_randint(seed, 10, 2 * t + 1, h->nx - 31);
  }
  // untrained network: all weights zero (predicts no change)
  if (hipMemsetAsync(S->at<float>(S->L.w), 0, (size_t)kSgNW * 4, h->stream) != hipSuccess ||
      hipMemsetAsync(S->at<float>(S->L.m), 0, (size_t)kSgNW * 4, h->stream) != hipSuccess ||
      hipMemsetAsync(S->at<float>(S->L.v), 0, (size_t)kSgNW * 4, h->stream) != hipSuccess ||
      hipMemsetAsync(S->at<long long>(S->L.counters), 0, 16, h->stream) != hipSuccess ||
      hipMemsetAsync(S->at<int>(S->L.flag), 0, 4, h->stream) != hipSuccess ||
      sg_repack(h) != hipSuccess) {
    err = "surrogate initialisation failed";
    return KB_EHIP;
  }
  return KB_OK;
}

void sg_destroy(kb_problem *h) {
  delete h->sg;
  h->sg = nullptr;
}

int sg_iter_depth(const kb_problem *h) { return h->sg->ksteps; }

int sg_kernels_per_block(const kb_problem *h) { return h->tile == 2 ? 8 : 3; }

// The k-step block, reading T[cur] and writing T[1-cur]:
//   fused (variant 0/1): network + check producers (1 kernel), check (1),
//                        predicated plain fallback (1);
//   per-layer (variant 2): input, 4 convolutions, check (2), fallback.
int sg_fill_iter(const kb_problem *h, int cur, Launch *L) {
  const SgState &S = *h->sg;
  const int H = (int)h->ny, W = (int)h->nx;
  const float *Tc = h->Tbuf[cur];
  float *Tn = h->Tbuf[1 - cur];
  const float *w = S.at<float>(S.L.w);
  SgCheckArgs k{};
  k.Tcur = Tc; k.Tnew = Tn; k.P = h->P; k.ny = H; k.nx = W; k.ksteps = S.ksteps; k.k = h->hk;
  for (int t = 0; t < 4; ++t) { k.tile_y[t] = S.tile_y[t]; k.tile_x[t] = S.tile_x[t]; }
  k.partial = S.at<double>(S.L.chk); k.plain = S.at<float>(S.L.plain);
  k.tail = SgCheckTail{S.at<double>(S.L.psum), std::pow(1.0 - (double)h->hk.cz, (double)S.ksteps), S.threshold,
                       S.at<int>(S.L.flag), S.at<double>(S.L.hist), kSgHistCap, S.at<long long>(S.L.counters)};
  int n = 0;
  if (h->tile != 2) {
    SgFusedArgs f{};
    f.T0 = Tc; f.P = h->P; f.Tout = Tn;
    f.w1 = S.at<unsigned short>(S.L.fwd1); f.w2 = S.at<unsigned short>(S.L.fwd2);
    f.w3 = S.at<unsigned short>(S.L.fwd3); f.w4 = S.at<unsigned short>(S.L.fwd4);
    f.bias = w; f.partial = k.partial; f.plain = k.plain; f.k = h->hk; f.s = S.s;
    f.H = H; f.W = W; f.tiles_x = S.tiles_x; f.ntiles = S.ntiles; f.nnet = S.nnet; f.ksteps = S.ksteps;
    for (int t = 0; t < 4; ++t) { f.tile_y[t] = S.tile_y[t]; f.tile_x[t] = S.tile_x[t]; }
    sg_make_fused(L[n++], f);
    k.nred = S.nnet;
    sg_make_check_final(L[n++], k);
  } else {
    unsigned short *x = S.at<unsigned short>(S.L.x);
    unsigned short *A0 = S.at<unsigned short>(S.L.act[0]), *A1 = S.at<unsigned short>(S.L.act[1]);
    sg_make_input(L[n++], SgInputArgs{Tc, h->P, x, S.n});
    SgConvArgs c{};
    c.npix = S.n; c.H = H; c.W = W; c.s = S.s;
    c.in = x; c.w = S.at<unsigned short>(S.L.fwd1); c.bias = w + kSgOffB[0]; c.out = A0;
    sg_make_conv(L[n++], c, 0);
    c.in = A0; c.w = S.at<unsigned short>(S.L.fwd2); c.bias = w + kSgOffB[1]; c.out = A1;
    sg_make_conv(L[n++], c, 1);
    c.in = A1; c.w = S.at<unsigned short>(S.L.fwd3); c.bias = w + kSgOffB[2]; c.out = A0;
    sg_make_conv(L[n++], c, 2);
    c.in = A0; c.w = S.at<unsigned short>(S.L.fwd4); c.bias = w + kSgOffB[3]; c.out = nullptr;
    c.T0 = Tc; c.Tout = Tn;
    sg_make_conv(L[n++], c, 3);
    k.nred = kSgRedBlocks;
    sg_make_check(L[n], L[n + 1], k);
    n += 2;
  }
  // fallback: the k plain steps in one predicated launch of the register
  // strips over 32x32 tiles (512 threads per block; a predicated-off launch
  // of the 64x16 LDS tiles, 1024 threads per block, costs more)
  Heat2DArgs f{Tc, Tn, h->P, H, W, h->hk, S.ksteps, S.at<int>(S.L.flag)};
  if (!make_heat2d_strip(L[n++], f, 23)) return -1;
  return n;
}

bool sg_field(const kb_problem *h, int field, float **dev, size_t *bytes) {
  const SgState &S = *h->sg;
  switch (field) {
    case KB_F_W: *dev = S.at<float>(S.L.w); *bytes = (size_t)kSgNW * 4; return true;
    case KB_F_SGSTATS: *dev = S.at<float>(S.L.counters); *bytes = 16; return true;
    case KB_F_RESID: *dev = S.at<float>(S.L.hist); *bytes = (size_t)kSgHistCap * 8; return true;
  }
  // the tape of the last training batch (read only)
  const size_t m = (size_t)S.last_m;
  if (m == 0 || field < KB_F_SG_X || field > KB_F_SG_GRAD) return false;
  switch (field) {
    case KB_F_SG_X: *dev = S.at<float>(S.L.xt); *bytes = m * 4; return true;
    case KB_F_SG_A1: case KB_F_SG_A2: case KB_F_SG_A3:
      *dev = S.at<float>(S.L.a[field - KB_F_SG_A1]); *bytes = m * 64; return true;
    case KB_F_SG_Z1: case KB_F_SG_Z2: case KB_F_SG_Z3:
      *dev = S.at<float>(S.L.z[field - KB_F_SG_Z1]); *bytes = m * 128; return true;
    case KB_F_SG_Y: *dev = S.at<float>(S.L.yt); *bytes = m * 4; return true;
    case KB_F_SG_TGT: *dev = S.at<float>(S.L.tgt); *bytes = m * 4; return true;
    case KB_F_SG_G4: *dev = S.at<float>(S.L.g4); *bytes = m * 4; return true;
    case KB_F_SG_G1: case KB_F_SG_G2: case KB_F_SG_G3:
      *dev = S.at<float>(S.L.g[field - KB_F_SG_G1]); *bytes = m * 128; return true;
    case KB_F_SG_GRAD: *dev = S.at<float>(S.L.grad); *bytes = (size_t)kSgNW * 4; return true;
  }
  return false;
}

}  // namespace kb

namespace {

int sg_fail(int code, const char *msg) { return kb_set_error(code, msg); }

#define SGCHK(expr)                                                       \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) return kb_set_error(KB_EHIP, hipGetErrorString(e_)); \
  } while (0)

// Forward + loss + backward on a batch of crops; leaves the gradient in
// the workspace.  Returns a KB status.
int sg_backprop(kb_problem *h, const float *T0, const float *P, const float *T16, int nfield, int Hf, int Wf,
                const int *crops, int ncrop, int C) {
  if (!h || !h->sg) return sg_fail(KB_EINVAL, "not a surrogate problem");
  SgState &S = *h->sg;
  if (!T0 || !P || !T16 || !crops || nfield < 1 || ncrop < 1 || ncrop > kSgMaxCrops || C < 64 || C % 64)
    return sg_fail(KB_EINVAL, "bad batch: need device fields, 1..1024 crops, crop size a multiple of 64");
  if ((long long)ncrop * C * C > S.train_pix) return sg_fail(KB_EINVAL, "batch exceeds the training capacity");
  for (int i = 0; i < ncrop; ++i) {
    const int f = crops[3 * i], y0 = crops[3 * i + 1], x0 = crops[3 * i + 2];
    if (f < 0 || f >= nfield || y0 < 0 || x0 < 0 || y0 + C > Hf || x0 + C > Wf)
      return sg_fail(KB_EINVAL, "crop outside its field");
  }
  hipStream_t st = h->stream;
  const long long m = (long long)ncrop * C * C;
  S.last_m = 0;
  int *crops_d = S.at<int>(S.L.crops);
  SGCHK(hipMemcpyAsync(crops_d, crops, (size_t)ncrop * 3 * 4, hipMemcpyHostToDevice, st));
  float *T0c = S.at<float>(S.L.T0c), *Pc = S.at<float>(S.L.Pc), *tgt = S.at<float>(S.L.tgt);
  SGCHK(sg_launch_crop(SgCropArgs{T0, P, T16, crops_d, T0c, Pc, tgt, ncrop, C, Hf, Wf, S.s}, st));
  unsigned short *xt = S.at<unsigned short>(S.L.xt);
  SGCHK(sg_launch_input(SgInputArgs{T0c, Pc, xt, m}, st));
  const float *w = S.at<float>(S.L.w);
  const unsigned short *fw[4] = {S.at<unsigned short>(S.L.fwd1), S.at<unsigned short>(S.L.fwd2),
                                 S.at<unsigned short>(S.L.fwd3), S.at<unsigned short>(S.L.fwd4)};
  const unsigned short *inp[4] = {xt, S.at<unsigned short>(S.L.a[0]), S.at<unsigned short>(S.L.a[1]),
                                  S.at<unsigned short>(S.L.a[2])};
  float *yt = S.at<float>(S.L.yt);
  for (int l = 0; l < 4; ++l) {
    SgConvArgs c{};
    c.npix = m; c.H = C; c.W = C; c.s = S.s;
    c.in = inp[l]; c.w = fw[l]; c.bias = w + kSgOffB[l];
    if (l < 3) { c.z = S.at<float>(S.L.z[l]); c.out = S.at<unsigned short>(S.L.a[l]); }
    else c.y = yt;
    Launch L;
    sg_make_conv(L, c, l);
    SGCHK(hipLaunchKernel(L.func, L.grid, L.block, L.params(), 0, st));
  }
  float *g4 = S.at<float>(S.L.g4);
  SGCHK(sg_launch_loss(SgLossArgs{yt, tgt, g4, S.at<double>(S.L.lossp), (float)m, m}, kSgLossBlocks, (double)m,
                       S.at<double>(S.L.loss), st));
  float *grad = S.at<float>(S.L.grad);
  const unsigned short *bw[4] = {nullptr, S.at<unsigned short>(S.L.bwd2), S.at<unsigned short>(S.L.bwd3),
                                 S.at<unsigned short>(S.L.bwd4)};
  const float *gl = g4;            // gradient of layer l's output
  for (int l = 3; l >= 0; --l) {
    const int cin = kSgCin[l], cout = kSgCout[l];
    SGCHK(sg_launch_wgrad(SgWgradArgs{gl, inp[l], S.at<float>(S.L.pw), S.at<float>(S.L.pb), ncrop, C, C}, cin,
                          cout, kSgWgradBlocks, st));
    SGCHK(sg_launch_reduce(SgReduceArgs{S.at<float>(S.L.pw), S.at<float>(S.L.pb), grad + kSgOffW[l],
                                        grad + kSgOffB[l], kSgWgradBlocks, cin, cout},
                           st));
    if (l == 0) break;
    float *gout = S.at<float>(S.L.g[l - 1]);   // dL/dz of layer l's input (kept for the tape)
    SGCHK(sg_launch_dgrad(SgDgradArgs{gl, bw[l], S.at<float>(S.L.z[l - 1]), gout, m, C, C}, cout, st));
    gl = gout;
  }
  S.last_m = m;
  return KB_OK;
}

}  // namespace

extern "C" {

int kb_sg_loss_grad(kb_problem *h, const float *T0, const float *P, const float *T16, int nfield, int Hf, int Wf,
                    const int *crops, int ncrop, int crop, double *loss, float *grad) {
  int rc = sg_backprop(h, T0, P, T16, nfield, Hf, Wf, crops, ncrop, crop);
  if (rc != KB_OK) return rc;
  SgState &S = *h->sg;
  SGCHK(hipStreamSynchronize(h->stream));
  if (loss) SGCHK(hipMemcpy(loss, S.at<double>(S.L.loss), 8, hipMemcpyDeviceToHost));
  if (grad) SGCHK(hipMemcpy(grad, S.at<float>(S.L.grad), (size_t)kSgNW * 4, hipMemcpyDeviceToHost));
  return KB_OK;
}

int kb_sg_train_step(kb_problem *h, const float *T0, const float *P, const float *T16, int nfield, int Hf, int Wf,
                     const int *crops, int ncrop, int crop, double lr, double *loss) {
  if (!(lr > 0)) return sg_fail(KB_EINVAL, "learning rate must be > 0");
  int rc = sg_backprop(h, T0, P, T16, nfield, Hf, Wf, crops, ncrop, crop);
  if (rc != KB_OK) return rc;
  SgState &S = *h->sg;
  S.adam_t += 1;
  const double b1 = 0.9, b2 = 0.999;
  SgAdamArgs a{S.at<float>(S.L.w), S.at<float>(S.L.m), S.at<float>(S.L.v), S.at<float>(S.L.grad),
               (float)lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, (double)S.adam_t)),
               (float)(1.0 - std::pow(b2, (double)S.adam_t)), kSgNW};
  SGCHK(sg_launch_adam(a, h->stream));
  SGCHK(sg_repack(h));
  if (loss) {
    SGCHK(hipMemcpyAsync(loss, S.at<double>(S.L.loss), 8, hipMemcpyDeviceToHost, h->stream));
    SGCHK(hipStreamSynchronize(h->stream));
  }
  return KB_OK;
}

}  // extern "C"
