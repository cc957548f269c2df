// Seeded initial state, the skeleton chain and the deterministic reductions.
#include <mutex>

#include "kb_internal.h"

namespace kb {

// ---------------------------------------------------------------------------
// Initial state: out[i] = float(lo + span * u), u = (z >> 40) * 2^-24 with
// z = splitmix(seed, tag, offset + i).  The double multiply and add are
// explicitly unfused so the host generator gives identical bits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_uniform_kernel(const InitArgs a) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t z = splitmix(a.seed, a.tag, a.offset + (uint64_t)i);
  const double u = (double)(z >> 40) * 0x1.0p-24;
  a.out[i] = (float)__dadd_rn(a.lo, __dmul_rn(a.span, u));
}

void make_init(Launch &L, const InitArgs &a) {
  L.set((const void *)init_uniform_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, a);
}

// ---------------------------------------------------------------------------
// Hot-spot power map (the surrogate workload's inputs): per cell
//   p = u + sum_h amp_h exp(-((y - cy_h)^2 + (x - cx_h)^2) / ((2 sigma_h) sigma_h))
// in double, each operation rounded once in this order, then one rounding
// to float; u is the cell's uniform draw of stream kTagP.  The spot count
// (1 + an integer draw on [0, 4)) and each spot's centre row, centre
// column, amplitude U[1,4) and width sigma U[4,32) are draws 0 and
// 1 + 4h .. 4 + 4h of stream kTagHot.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hot_spot_kernel(const HotSpotArgs a) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)a.ny * a.nx) return;
  const int y = (int)(i / a.nx), x = (int)(i - (long long)y * a.nx);
  const uint64_t z = splitmix(a.seed, kTagP, (uint64_t)i);
  double p = (double)(z >> 40) * 0x1.0p-24;
  for (int h = 0; h < a.count; ++h) {
    const double dy = __dsub_rn((double)y, a.cy[h]), dx = __dsub_rn((double)x, a.cx[h]);
    const double r2 = __dadd_rn(__dmul_rn(dy, dy), __dmul_rn(dx, dx));
    p = __dadd_rn(p, __dmul_rn(a.amp[h], exp(-__ddiv_rn(r2, a.den[h]))));
  }
  a.out[i] = (float)p;
}

void make_hot_spots(Launch &L, const HotSpotArgs &a) {
  const long long n = (long long)a.ny * a.nx;
  L.set((const void *)hot_spot_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, a);
}

static double host_u01(uint64_t seed, uint64_t tag, uint64_t idx) {
  return (double)(splitmix(seed, tag, idx) >> 40) * 0x1.0p-24;
}

HotSpotArgs host_hot_spots(float *out, int ny, int nx, uint64_t seed) {
  HotSpotArgs a{};
  a.out = out; a.ny = ny; a.nx = nx; a.seed = seed;
  a.count = 1 + (int)host_randint(seed, kTagHot, 0, 4);
  for (int h = 0; h < a.count; ++h) {
    const double u0 = host_u01(seed, kTagHot, 1 + 4 * h), u1 = host_u01(seed, kTagHot, 2 + 4 * h);
    const double u2 = host_u01(seed, kTagHot, 3 + 4 * h), u3 = host_u01(seed, kTagHot, 4 + 4 * h);
    const double sig = 4.0 + 28.0 * u3;            // built with -ffp-contract=off: no fusion
    a.cy[h] = u0 * ny;
    a.cx[h] = u1 * nx;
    a.amp[h] = 1.0 + 3.0 * u2;
    a.den[h] = 2.0 * sig * sig;
  }
  return a;
}

float host_uniform(uint64_t seed, uint64_t tag, uint64_t idx, double lo, double hi) {
  const uint64_t z = splitmix(seed, tag, idx);
  const double u = (double)(z >> 40) * 0x1.0p-24;
  return (float)(lo + (hi - lo) * u);   // built with -ffp-contract=off: no fusion
}

int64_t host_randint(uint64_t seed, uint64_t tag, uint64_t idx, int64_t m) {
  const uint64_t top = splitmix(seed, tag, idx) >> 40;
  return (int64_t)((top * (uint64_t)m) >> 24);
}

// ---------------------------------------------------------------------------
// Skeleton kernel: x <- fma(a, x, b) on every element (the skeleton
// application's small element-wise kernel, Sec. III-C).  Memory-bound at
// 8 bytes per element; variant picks elements per thread.
// ---------------------------------------------------------------------------
template <int VEC>
__global__ __launch_bounds__(256) void skeleton_kernel(const SkelArgs s) {
  const long long base = ((long long)blockIdx.x * 256 + threadIdx.x) * VEC;
  if (base + VEC <= s.n) {
    if constexpr (VEC == 4) {
      float4 v = *reinterpret_cast<const float4 *>(s.x + base);
      v.x = fmaf(s.a, v.x, s.b);
      v.y = fmaf(s.a, v.y, s.b);
      v.z = fmaf(s.a, v.z, s.b);
      v.w = fmaf(s.a, v.w, s.b);
      *reinterpret_cast<float4 *>(s.x + base) = v;
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) s.x[base + e] = fmaf(s.a, s.x[base + e], s.b);
    }
  } else {
    for (long long e = base; e < s.n; ++e) s.x[e] = fmaf(s.a, s.x[e], s.b);
  }
}

// variant: 1 = 4 elements per thread (16-byte access), 2 = 1 element, 3 = 8
void make_skeleton(Launch &L, const SkelArgs &a, int variant) {
  int vec = variant == 2 ? 1 : (variant == 3 ? 8 : 4);
  long long threads = (a.n + vec - 1) / vec;
  dim3 grid((unsigned)((threads + 255) / 256));
  if (vec == 1) L.set((const void *)skeleton_kernel<1>, grid, dim3(256), 0, a);
  else if (vec == 8) L.set((const void *)skeleton_kernel<8>, grid, dim3(256), 0, a);
  else L.set((const void *)skeleton_kernel<4>, grid, dim3(256), 0, a);
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Pass 1: block b sums a fixed contiguous chunk
// (each thread a fixed strided subset, in double), then a fixed wave64
// butterfly and a fixed cross-wave order; pass 2: one block sums the
// partials the same way.  The result depends only on n, never on timing.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
int reduce_max_blocks() { return kRedBlocks; }

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[4];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
  return r;
}

struct RedArgs {
  const float *f[6]; int nf; int square; long long n; long long chunk; double *partials;
};

__global__ __launch_bounds__(256) void reduce_pass1(const RedArgs a) {
  const long long lo = (long long)blockIdx.x * a.chunk;
  const long long hi = min(lo + a.chunk, a.n);
  double acc = 0.0;
  for (int q = 0; q < a.nf; ++q) {
    const float *x = a.f[q];
    for (long long i = lo + threadIdx.x; i < hi; i += 256) {
      const double v = (double)x[i];
      acc += a.square ? v * v : v;
    }
  }
  const double r = block_sum(acc);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void reduce_pass2(const double *partials, int nb, double *out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partials[i];
  const double r = block_sum(acc);
  if (threadIdx.x == 0) *out = r;
}

// In-chain reductions (see RedLogArgs).  Pass 1: grid (nb, ngroups).
__global__ __launch_bounds__(256) void reduce_log_pass1(const RedLogArgs a) {
  const int g = blockIdx.y, per = a.nf / a.ngroups;
  const long long lo = (long long)blockIdx.x * a.chunk;
  const long long hi = min(lo + a.chunk, a.n);
  double acc = 0.0;
  for (int q = 0; q < per; ++q) {
    const float *x = a.f[g * per + q];
    for (long long i = lo + threadIdx.x; i < hi; i += 256) {
      const double v = (double)x[i];
      acc += a.square ? v * v : v;
    }
  }
  const double r = block_sum(acc);
  if (threadIdx.x == 0) a.partials[g * a.nb + blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void reduce_log_pass2(const RedLogArgs a) {
  double v[2] = {0.0, 0.0};
  for (int g = 0; g < a.ngroups; ++g) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < a.nb; i += 256) acc += a.partials[g * a.nb + i];
    v[g] = block_sum(acc);
    __syncthreads();                       // block_sum's LDS is reused
  }
  if (threadIdx.x == 0) {
    const long long c = *a.count;
    if (c >= 0 && c < a.cap) {
      double *e = a.log + c * 4;
      e[0] = (double)((c + 1) * a.every);
      e[1] = v[0];
      e[2] = v[1];
      e[3] = 0.0;
    }
    *a.count = c + 1;
  }
}

RedLogArgs reduce_log_args(const float *const *fields, int nf, int ngroups, int square, long long n, double *partials,
                           double *log, long long *count, long long every) {
  RedLogArgs a{};
  for (int q = 0; q < nf && q < 6; ++q) a.f[q] = fields[q];
  long long chunk = (n + kRedBlocks - 1) / kRedBlocks;
  chunk = ((chunk + 1023) / 1024) * 1024;
  if (chunk < 1024) chunk = 1024;
  a.nf = nf; a.ngroups = ngroups; a.square = square; a.n = n; a.chunk = chunk;
  a.nb = n > 0 ? (int)((n + chunk - 1) / chunk) : 1;
  a.partials = partials; a.log = log; a.count = count; a.cap = kRedLogCap; a.every = every;
  return a;
}

void make_reduce_log(Launch &L1, Launch &L2, const RedLogArgs &a) {
  L1.set((const void *)reduce_log_pass1, dim3(a.nb, a.ngroups), dim3(256), 0, a);
  L2.set((const void *)reduce_log_pass2, dim3(1), dim3(256), 0, a);
}

hipError_t reduce_impl(const float *const *f, int nf, int square, long long n, double *partials, double *result,
                       hipStream_t s) {
  long long chunk = (n + kRedBlocks - 1) / kRedBlocks;
  chunk = ((chunk + 1023) / 1024) * 1024;
  if (chunk < 1024) chunk = 1024;
  const int nb = n > 0 ? (int)((n + chunk - 1) / chunk) : 1;
  RedArgs a{};
  for (int q = 0; q < nf && q < 6; ++q) a.f[q] = f[q];
  a.nf = nf; a.square = square; a.n = n; a.chunk = chunk; a.partials = partials;
  hipLaunchKernelGGL(reduce_pass1, dim3(nb), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(256), 0, s, (const double *)partials, nb, result);
  return hipGetLastError();
}

hipError_t reduce_sum(const float *x, long long n, double *partials, double *result, hipStream_t s) {
  const float *f[1] = {x};
  return reduce_impl(f, 1, 0, n, partials, result, s);
}

hipError_t reduce_sumsq(const float *const *fields, int nf, long long n, double *partials, double *result,
                        hipStream_t s) {
  return reduce_impl(fields, nf, 1, n, partials, result, s);
}

}  // namespace kb

// ---------------------------------------------------------------------------
// The reduction without a workspace (kb_reduce_noalloc): the per-block
// partials live in this file-scope device array, one copy per GPU, held
// until the process ends (kRedBlocks doubles = 8 KiB).  Host code never
// passes the array's name to a kernel: the name is a host-side stand-in.
// Its device address is resolved once per device with hipGetSymbolAddress
// and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kb::kRedBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device (resolved on the first call
// there); nullptr and a message on failure.
double *scratch_on_current_device(const char **why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *why = "no current HIP device (or device index >= 64)";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = "hipGetSymbolAddress of the scratch array failed";
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int kb_reduce_noalloc(const float *const *x, int nx, int64_t n, int square, double *out, void *stream) {
  if (!x || !out || nx < 1 || nx > 6 || n < 0 || (square != 0 && square != 1))
    return kb::kb_set_error(KB_EINVAL, "kb_reduce_noalloc: need 1..6 arrays, n >= 0, square 0 or 1, an output");
  if (n > kb::kReduceNoallocMaxN)
    return kb::kb_set_error(KB_EINVAL, "kb_reduce_noalloc: n exceeds the 2^40 elements per array it accepts");
  for (int q = 0; q < nx; ++q)
    if (!x[q] && n > 0) return kb::kb_set_error(KB_EINVAL, "kb_reduce_noalloc: null array");
  const char *why = "";
  double *partials = scratch_on_current_device(&why);
  if (!partials) return kb::kb_set_error(KB_EHIP, why);
  const hipError_t e = kb::reduce_impl(x, nx, square, n, partials, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return kb::kb_set_error(KB_EHIP, hipGetErrorString(e));
  return KB_OK;
}

namespace kb {

// ---------------------------------------------------------------------------
// Streaming calibration: out_j[i] = sum_k in_k[i], one float4 i per thread
// over a full grid (the launch shape of the stencil kernels).  Used only to
// measure the DRAM throughput a given number of concurrent read / write
// streams reaches.
// ---------------------------------------------------------------------------
struct StreamArgs {
  const float4 *in[8];
  float4 *out[8];
  int nin, nout;
  long long n4;
};

__global__ __launch_bounds__(256) void stream_probe_kernel(const StreamArgs a) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n4) return;
  float4 v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < a.nin) v[k] = a.in[k][i];            // all loads in flight before the sum
  float4 s = v[0];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (k < a.nin) { s.x += v[k].x; s.y += v[k].y; s.z += v[k].z; s.w += v[k].w; }
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < a.nout) a.out[j][i] = s;
}

hipError_t stream_probe(int nin, int nout, long long n, float *ws, hipStream_t s, int reps, double *seconds) {
  StreamArgs a{};
  for (int k = 0; k < nin; ++k) a.in[k] = reinterpret_cast<const float4 *>(ws + (size_t)k * n);
  for (int j = 0; j < nout; ++j) a.out[j] = reinterpret_cast<float4 *>(ws + (size_t)(nin + j) * n);
  a.nin = nin; a.nout = nout; a.n4 = n / 4;
  const long long blocks = (a.n4 + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipError_t e;
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return e; }
  hipLaunchKernelGGL(stream_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    hipLaunchKernelGGL(stream_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) *seconds = ms * 1e-3 / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace kb
