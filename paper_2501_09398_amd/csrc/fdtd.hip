// Yee FDTD kernels for the PEC cavity (the FDTD Maxwell solver of Sec. III-C:
// an H kernel and an E kernel per step, plus the soft-source kernel).
//
// dx = 1, eps = mu = 1.  Each field lives on (N+1)^3 nodes stored with a row
// pitch P (a multiple of 4 floats >= N+1, so every row starts on a 16-byte
// boundary): node (i, j, k) is at (k*(N+1) + j)*P + i; the columns i > N are
// padding and stay zero.  Component positions:
//   Ex(i+1/2, j, k)  Ey(i, j+1/2, k)  Ez(i, j, k+1/2)
//   Hx(i, j+1/2, k+1/2)  Hy(i+1/2, j, k+1/2)  Hz(i+1/2, j+1/2, k)
// H -= dt * curl E on every H node (Hx for i <= N, j, k < N; Hy for i, k < N;
// Hz for i, j < N); E += dt * curl H on the interior E nodes only, so the
// tangential E on the walls is never written (PEC).  Each update is
// new = old -/+ dt*((a - b) - (c - d)) with that exact grouping; dt = 0.5
// makes the product exact, so fused and unfused evaluation agree.
//
// Both kernels are HBM-bound: 36 algorithmic bytes per node (three fields
// read, three read and written).
#include <algorithm>

#include "kb_internal.h"

namespace kb {

// ---------------------------------------------------------------------------
// Scalar kernels: one thread per node, 64x4 threads over (i, j), grid z = k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fdtd_h_kernel(const FdtdArgs f) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  const int N = f.N;
  if (i > N || j > N) return;
  const long long M = N + 1;
  const long long sj = f.P, sk = M * f.P;
  const long long c = (long long)k * sk + (long long)j * sj + i;
  const float dt = f.dt;
  if (j < N && k < N)
    f.Hx[c] = f.Hx[c] - dt * ((f.Ez[c + sj] - f.Ez[c]) - (f.Ey[c + sk] - f.Ey[c]));
  if (i < N && k < N)
    f.Hy[c] = f.Hy[c] - dt * ((f.Ex[c + sk] - f.Ex[c]) - (f.Ez[c + 1] - f.Ez[c]));
  if (i < N && j < N)
    f.Hz[c] = f.Hz[c] - dt * ((f.Ey[c + 1] - f.Ey[c]) - (f.Ex[c + sj] - f.Ex[c]));
}

__global__ __launch_bounds__(256) void fdtd_e_kernel(const FdtdArgs f) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  const int N = f.N;
  if (i > N || j > N) return;
  const long long M = N + 1;
  const long long sj = f.P, sk = M * f.P;
  const long long c = (long long)k * sk + (long long)j * sj + i;
  const float dt = f.dt;
  const bool ii = i >= 1 && i <= N - 1;
  const bool jj = j >= 1 && j <= N - 1;
  const bool kk = k >= 1 && k <= N - 1;
  if (i < N && jj && kk)
    f.Ex[c] = f.Ex[c] + dt * ((f.Hz[c] - f.Hz[c - sj]) - (f.Hy[c] - f.Hy[c - sk]));
  if (j < N && ii && kk)
    f.Ey[c] = f.Ey[c] + dt * ((f.Hx[c] - f.Hx[c - sk]) - (f.Hz[c] - f.Hz[c - 1]));
  if (k < N && ii && jj)
    f.Ez[c] = f.Ez[c] + dt * ((f.Hy[c] - f.Hy[c - 1]) - (f.Hx[c] - f.Hx[c - sj]));
}

static dim3 scalar_grid(int N) {
  return dim3((unsigned)((N + 1 + 63) / 64), (unsigned)((N + 1 + 3) / 4), (unsigned)(N + 1));
}

// ---------------------------------------------------------------------------
// Vector kernels: one thread per float4 of four consecutive nodes in i.  A
// plane's float4 slots are numbered q = j*(P/4) + i/4 and split into blocks
// of 256; blocks are numbered plane by plane and remapped so that each XCD
// runs one contiguous band of planes, keeping the k+1 (H) or k-1 (E) plane a
// block reads in the same L2 as the block that owns it.  Neighbours along i
// come from the adjacent lane (wave shuffle) or, at a wave edge, from
// memory; along j and k from memory (cache).  Components whose node is not
// updated keep their old value, so the float4 store rewrites them unchanged.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, const float4 &v) { *reinterpret_cast<float4 *>(p) = v; }
__device__ __forceinline__ float comp(const float4 &v, int e) {
  return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

struct VecPos {
  int k, j, i0, lane;
  bool qin;
  size_t c;        // offset of node (i0, j, k)
};

__device__ __forceinline__ bool vec_pos(const FdtdArgs &f, VecPos &p) {
  const int M = f.N + 1, P4 = f.P / 4;
  const int Q = M * P4;                       // float4 slots per plane
  const int bpp = (Q + 255) / 256;            // blocks per plane
  const int nb = bpp * M;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return false;
  p.k = lb / bpp;
  const int q = (lb - p.k * bpp) * 256 + (int)threadIdx.x;
  p.qin = q < Q;
  const int qq = p.qin ? q : Q - 1;
  p.j = qq / P4;
  p.i0 = (qq - p.j * P4) * 4;
  p.lane = threadIdx.x & 63;
  p.c = ((size_t)p.k * M + p.j) * f.P + p.i0;
  return true;
}

__global__ __launch_bounds__(256) void fdtd_h_vec_kernel(const FdtdArgs f) {
  VecPos p;
  if (!vec_pos(f, p)) return;
  const int N = f.N;
  const size_t sj = f.P, sk = (size_t)(N + 1) * f.P;
  const float *__restrict__ Ex = f.Ex;
  const float *__restrict__ Ey = f.Ey;
  const float *__restrict__ Ez = f.Ez;
  float *__restrict__ Hx = f.Hx;
  float *__restrict__ Hy = f.Hy;
  float *__restrict__ Hz = f.Hz;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const size_t c = p.c;
  const bool in = p.qin;
  const float4 ex = in ? ld4(Ex + c) : z4;
  const float4 ey = in ? ld4(Ey + c) : z4;
  const float4 ez = in ? ld4(Ez + c) : z4;
  const float4 hx = in ? ld4(Hx + c) : z4;
  const float4 hy = in ? ld4(Hy + c) : z4;
  const float4 hz = in ? ld4(Hz + c) : z4;
  const bool kup = in && p.k < N, jup = in && p.j < N;
  const float4 ex_k = kup ? ld4(Ex + c + sk) : z4;     // k+1
  const float4 ey_k = kup ? ld4(Ey + c + sk) : z4;
  const float4 ez_j = jup ? ld4(Ez + c + sj) : z4;     // j+1
  const float4 ex_j = jup ? ld4(Ex + c + sj) : z4;
  // i+4 (east of the last component): the next lane's first component when
  // it is in the same row, else memory; past the row it is never used.
  float ey_e = lane_east_open(ey.x);
  float ez_e = lane_east_open(ez.x);
  if (p.lane == 63 && in && p.i0 + 4 < f.P) {
    ey_e = Ey[c + 4];
    ez_e = Ez[c + 4];
  }
  const float dt = f.dt;
  float ox[4], oy[4], oz[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = p.i0 + e;
    const float eyc = comp(ey, e), ezc = comp(ez, e), exc = comp(ex, e);
    const float eye = e < 3 ? comp(ey, e + 1) : ey_e;
    const float eze = e < 3 ? comp(ez, e + 1) : ez_e;
    ox[e] = (i <= N && p.j < N && p.k < N)
                ? comp(hx, e) - dt * ((comp(ez_j, e) - ezc) - (comp(ey_k, e) - eyc)) : comp(hx, e);
    oy[e] = (i < N && p.k < N) ? comp(hy, e) - dt * ((comp(ex_k, e) - exc) - (eze - ezc)) : comp(hy, e);
    oz[e] = (i < N && p.j < N) ? comp(hz, e) - dt * ((eye - eyc) - (comp(ex_j, e) - exc)) : comp(hz, e);
  }
  if (in) {
    st4(Hx + c, make_float4(ox[0], ox[1], ox[2], ox[3]));
    st4(Hy + c, make_float4(oy[0], oy[1], oy[2], oy[3]));
    st4(Hz + c, make_float4(oz[0], oz[1], oz[2], oz[3]));
  }
}

__global__ __launch_bounds__(256) void fdtd_e_vec_kernel(const FdtdArgs f) {
  VecPos p;
  if (!vec_pos(f, p)) return;
  const int N = f.N;
  const size_t sj = f.P, sk = (size_t)(N + 1) * f.P;
  float *__restrict__ Ex = f.Ex;
  float *__restrict__ Ey = f.Ey;
  float *__restrict__ Ez = f.Ez;
  const float *__restrict__ Hx = f.Hx;
  const float *__restrict__ Hy = f.Hy;
  const float *__restrict__ Hz = f.Hz;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const size_t c = p.c;
  const bool in = p.qin;
  const float4 ex = in ? ld4(Ex + c) : z4;
  const float4 ey = in ? ld4(Ey + c) : z4;
  const float4 ez = in ? ld4(Ez + c) : z4;
  const float4 hx = in ? ld4(Hx + c) : z4;
  const float4 hy = in ? ld4(Hy + c) : z4;
  const float4 hz = in ? ld4(Hz + c) : z4;
  const bool kdn = in && p.k > 0, jdn = in && p.j > 0;
  const float4 hy_k = kdn ? ld4(Hy + c - sk) : z4;     // k-1
  const float4 hx_k = kdn ? ld4(Hx + c - sk) : z4;
  const float4 hz_j = jdn ? ld4(Hz + c - sj) : z4;     // j-1
  const float4 hx_j = jdn ? ld4(Hx + c - sj) : z4;
  // i-1 (west of the first component): the previous lane's last component
  // when it is in the same row, else memory; at i = 0 it is never used.
  float hz_w = lane_west_open(hz.w);
  float hy_w = lane_west_open(hy.w);
  if (p.lane == 0 && in && p.i0 > 0) {
    hz_w = Hz[c - 1];
    hy_w = Hy[c - 1];
  }
  const float dt = f.dt;
  const bool jj = p.j >= 1 && p.j <= N - 1;
  const bool kk = p.k >= 1 && p.k <= N - 1;
  float ox[4], oy[4], oz[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = p.i0 + e;
    const bool ii = i >= 1 && i <= N - 1;
    const float hzc = comp(hz, e), hyc = comp(hy, e), hxc = comp(hx, e);
    const float hzw = e > 0 ? comp(hz, e - 1) : hz_w;
    const float hyw = e > 0 ? comp(hy, e - 1) : hy_w;
    ox[e] = (i < N && jj && kk) ? comp(ex, e) + dt * ((hzc - comp(hz_j, e)) - (hyc - comp(hy_k, e))) : comp(ex, e);
    oy[e] = (p.j < N && ii && kk) ? comp(ey, e) + dt * ((hxc - comp(hx_k, e)) - (hzc - hzw)) : comp(ey, e);
    oz[e] = (p.k < N && ii && jj) ? comp(ez, e) + dt * ((hyc - hyw) - (hxc - comp(hx_j, e))) : comp(ez, e);
  }
  if (in) {
    st4(Ex + c, make_float4(ox[0], ox[1], ox[2], ox[3]));
    st4(Ey + c, make_float4(oy[0], oy[1], oy[2], oy[3]));
    st4(Ez + c, make_float4(oz[0], oz[1], oz[2], oz[3]));
  }
}

// ---------------------------------------------------------------------------
// k-marching vector kernels: a thread owns one float4 slot of a plane for KC
// consecutive planes and walks them in increasing k, so the H kernel reuses
// the k+1 row of Ex, Ey it loaded as the next plane's own row and the E
// kernel the Hx, Hy it loaded as the next plane's k-1 row (8 float4 loads
// per node instead of 10).  Blocks are numbered by (plane chunk, slot block)
// and remapped to XCD bands as above.  Same arithmetic, same bits.
// ---------------------------------------------------------------------------
struct MarchPos {
  int k0, k1, j, i0, lane;
  bool qin;
  size_t c;        // offset of node (i0, j, k0)
};

template <int KC>
__device__ __forceinline__ bool march_pos(int N, int P, MarchPos &p) {
  const int M = N + 1, P4 = P / 4;
  const int Q = M * P4;
  const int bpp = (Q + 255) / 256;
  const int nch = (M + KC - 1) / KC;
  const int nb = bpp * nch;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return false;
  const int ch = lb / bpp;
  const int q = (lb - ch * bpp) * 256 + (int)threadIdx.x;
  p.qin = q < Q;
  const int qq = p.qin ? q : Q - 1;
  p.j = qq / P4;
  p.i0 = (qq - p.j * P4) * 4;
  p.lane = threadIdx.x & 63;
  p.k0 = ch * KC;
  p.k1 = min(p.k0 + KC, M);
  p.c = ((size_t)p.k0 * M + p.j) * P + p.i0;
  return true;
}

template <int KC>
__global__ __launch_bounds__(256) void fdtd_h_march_kernel(const FdtdArgs f) {
  MarchPos p;
  if (!march_pos<KC>(f.N, f.P, p)) return;
  const int N = f.N;
  const size_t sj = f.P, sk = (size_t)(N + 1) * f.P;
  const float *__restrict__ Ex = f.Ex;
  const float *__restrict__ Ey = f.Ey;
  const float *__restrict__ Ez = f.Ez;
  float *__restrict__ Hx = f.Hx;
  float *__restrict__ Hy = f.Hy;
  float *__restrict__ Hz = f.Hz;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const bool in = p.qin;
  const bool jup = in && p.j < N;
  const float dt = f.dt;
  size_t c = p.c;
  float4 ex = in ? ld4(Ex + c) : z4;
  float4 ey = in ? ld4(Ey + c) : z4;
  for (int k = p.k0; k < p.k1; ++k, c += sk) {
    const bool kup = in && k < N;
    const float4 ex_k = kup ? ld4(Ex + c + sk) : z4;   // k+1
    const float4 ey_k = kup ? ld4(Ey + c + sk) : z4;
    const float4 ez = in ? ld4(Ez + c) : z4;
    const float4 hx = in ? ld4(Hx + c) : z4;
    const float4 hy = in ? ld4(Hy + c) : z4;
    const float4 hz = in ? ld4(Hz + c) : z4;
    const float4 ez_j = jup ? ld4(Ez + c + sj) : z4;   // j+1
    const float4 ex_j = jup ? ld4(Ex + c + sj) : z4;
    float ey_e = lane_east_open(ey.x);
    float ez_e = lane_east_open(ez.x);
    if (p.lane == 63 && in && p.i0 + 4 < f.P) {
      ey_e = Ey[c + 4];
      ez_e = Ez[c + 4];
    }
    float ox[4], oy[4], oz[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = p.i0 + e;
      const float eyc = comp(ey, e), ezc = comp(ez, e), exc = comp(ex, e);
      const float eye = e < 3 ? comp(ey, e + 1) : ey_e;
      const float eze = e < 3 ? comp(ez, e + 1) : ez_e;
      ox[e] = (i <= N && p.j < N && k < N)
                  ? comp(hx, e) - dt * ((comp(ez_j, e) - ezc) - (comp(ey_k, e) - eyc)) : comp(hx, e);
      oy[e] = (i < N && k < N) ? comp(hy, e) - dt * ((comp(ex_k, e) - exc) - (eze - ezc)) : comp(hy, e);
      oz[e] = (i < N && p.j < N) ? comp(hz, e) - dt * ((eye - eyc) - (comp(ex_j, e) - exc)) : comp(hz, e);
    }
    if (in) {
      st4(Hx + c, make_float4(ox[0], ox[1], ox[2], ox[3]));
      st4(Hy + c, make_float4(oy[0], oy[1], oy[2], oy[3]));
      st4(Hz + c, make_float4(oz[0], oz[1], oz[2], oz[3]));
    }
    ex = ex_k;
    ey = ey_k;
  }
}

template <int KC>
__global__ __launch_bounds__(256) void fdtd_e_march_kernel(const FdtdArgs f) {
  MarchPos p;
  if (!march_pos<KC>(f.N, f.P, p)) return;
  const int N = f.N;
  const size_t sj = f.P, sk = (size_t)(N + 1) * f.P;
  float *__restrict__ Ex = f.Ex;
  float *__restrict__ Ey = f.Ey;
  float *__restrict__ Ez = f.Ez;
  const float *__restrict__ Hx = f.Hx;
  const float *__restrict__ Hy = f.Hy;
  const float *__restrict__ Hz = f.Hz;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const bool in = p.qin;
  const bool jdn = in && p.j > 0;
  const bool jj = p.j >= 1 && p.j <= N - 1;
  const float dt = f.dt;
  size_t c = p.c;
  float4 hx_k = in && p.k0 > 0 ? ld4(Hx + c - sk) : z4;   // k-1
  float4 hy_k = in && p.k0 > 0 ? ld4(Hy + c - sk) : z4;
  for (int k = p.k0; k < p.k1; ++k, c += sk) {
    const float4 ex = in ? ld4(Ex + c) : z4;
    const float4 ey = in ? ld4(Ey + c) : z4;
    const float4 ez = in ? ld4(Ez + c) : z4;
    const float4 hx = in ? ld4(Hx + c) : z4;
    const float4 hy = in ? ld4(Hy + c) : z4;
    const float4 hz = in ? ld4(Hz + c) : z4;
    const float4 hz_j = jdn ? ld4(Hz + c - sj) : z4;   // j-1
    const float4 hx_j = jdn ? ld4(Hx + c - sj) : z4;
    float hz_w = lane_west_open(hz.w);
    float hy_w = lane_west_open(hy.w);
    if (p.lane == 0 && in && p.i0 > 0) {
      hz_w = Hz[c - 1];
      hy_w = Hy[c - 1];
    }
    const bool kk = k >= 1 && k <= N - 1;
    float ox[4], oy[4], oz[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = p.i0 + e;
      const bool ii = i >= 1 && i <= N - 1;
      const float hzc = comp(hz, e), hyc = comp(hy, e), hxc = comp(hx, e);
      const float hzw = e > 0 ? comp(hz, e - 1) : hz_w;
      const float hyw = e > 0 ? comp(hy, e - 1) : hy_w;
      ox[e] = (i < N && jj && kk) ? comp(ex, e) + dt * ((hzc - comp(hz_j, e)) - (hyc - comp(hy_k, e))) : comp(ex, e);
      oy[e] = (p.j < N && ii && kk) ? comp(ey, e) + dt * ((hxc - comp(hx_k, e)) - (hzc - hzw)) : comp(ey, e);
      oz[e] = (k < N && ii && jj) ? comp(ez, e) + dt * ((hyc - hyw) - (hxc - comp(hx_j, e))) : comp(ez, e);
    }
    if (in) {
      st4(Ex + c, make_float4(ox[0], ox[1], ox[2], ox[3]));
      st4(Ey + c, make_float4(oy[0], oy[1], oy[2], oy[3]));
      st4(Ez + c, make_float4(oz[0], oz[1], oz[2], oz[3]));
    }
    hx_k = hx;
    hy_k = hy;
  }
}

template <int KC>
static dim3 march_grid(int N, int P) {
  const int M = N + 1, P4 = P / 4;
  const int bpp = (M * P4 + 255) / 256;
  return dim3((unsigned)xcd_padded_grid(bpp * ((M + KC - 1) / KC)));
}

static dim3 vec_grid(const FdtdArgs &a) {
  const int M = a.N + 1, P4 = a.P / 4;
  const int bpp = (M * P4 + 255) / 256;
  return dim3((unsigned)xcd_padded_grid(bpp * M));
}

// variant: 1 = scalar, 2 = vector (default), 3 / 4 = vector marching 8 / 16
// planes per thread
bool make_fdtd_h(Launch &L, const FdtdArgs &a, int variant) {
  if (variant == 1) L.set((const void *)fdtd_h_kernel, scalar_grid(a.N), dim3(64, 4), 0, a);
  else if (variant == 2) L.set((const void *)fdtd_h_vec_kernel, vec_grid(a), dim3(256), 0, a);
  else if (variant == 3) L.set((const void *)fdtd_h_march_kernel<8>, march_grid<8>(a.N, a.P), dim3(256), 0, a);
  else if (variant == 4) L.set((const void *)fdtd_h_march_kernel<16>, march_grid<16>(a.N, a.P), dim3(256), 0, a);
  else return false;
  return true;
}

bool make_fdtd_e(Launch &L, const FdtdArgs &a, int variant) {
  if (variant == 1) L.set((const void *)fdtd_e_kernel, scalar_grid(a.N), dim3(64, 4), 0, a);
  else if (variant == 2) L.set((const void *)fdtd_e_vec_kernel, vec_grid(a), dim3(256), 0, a);
  else if (variant == 3) L.set((const void *)fdtd_e_march_kernel<8>, march_grid<8>(a.N, a.P), dim3(256), 0, a);
  else if (variant == 4) L.set((const void *)fdtd_e_march_kernel<16>, march_grid<16>(a.N, a.P), dim3(256), 0, a);
  else return false;
  return true;
}

// ---------------------------------------------------------------------------
// Fused H + E kernel (variant 5): one launch per step reads E^n and H^{n-1/2}
// from one set of buffers and writes H^{n+1/2} and E^{n+1} to the other, so
// a node-step moves 48 bytes (six fields read, six written) instead of 72.
// A thread owns a float4 slot of a row and walks KC planes in increasing k
// (KC = 1: one plane).  The E update needs H^{n+1/2} at its own node and at
// i-1, j-1 and k-1: the own value is computed, the k-1 value is the
// previous plane's (recomputed from the old fields for the first plane),
// i-1 comes from the neighbouring lane (recomputed from memory by the first
// lane of a wave), and the j-1 row is recomputed from the old fields.  The
// extra loads hit L2 (the neighbouring rows and planes are other threads'
// own data); HBM sees each field read once and written once.  Every
// recomputed value uses the H kernel's formula and operand order, so it
// equals the owner's bit for bit, and the whole step equals the H kernel
// followed by the E kernel.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));

// Float4 store; NT = non-temporal (streaming) store that does not keep the
// line in cache, leaving L2 to the neighbouring rows and planes being read.
template <bool NT>
__device__ __forceinline__ void st4o(float *p, float a, float b, float c, float d) {
  if constexpr (NT) {
    f4v v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(p));
  } else {
    *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
  }
}

template <int KC, bool NT>
__global__ __launch_bounds__(256) void fdtd_fused_kernel(const FdtdFusedArgs f) {
  MarchPos p;
  if (!march_pos<KC>(f.N, f.P, p)) return;
  const int N = f.N;
  const size_t sj = f.P, sk = (size_t)(N + 1) * f.P;
  const float *__restrict__ Ex = f.Ex;
  const float *__restrict__ Ey = f.Ey;
  const float *__restrict__ Ez = f.Ez;
  const float *__restrict__ Hx = f.Hx;
  const float *__restrict__ Hy = f.Hy;
  const float *__restrict__ Hz = f.Hz;
  float *__restrict__ oEx = f.oEx;
  float *__restrict__ oEy = f.oEy;
  float *__restrict__ oEz = f.oEz;
  float *__restrict__ oHx = f.oHx;
  float *__restrict__ oHy = f.oHy;
  float *__restrict__ oHz = f.oHz;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const bool in = p.qin;
  const int j = p.j;
  const bool jup = in && j < N, jdn = in && j > 0;
  const bool jj = j >= 1 && j <= N - 1;
  const float dt = f.dt;
  size_t c = p.c;
  // E^n at (j, k0) and, for the j-1 row, Ey^n at (j-1, k0)
  float4 ex = in ? ld4(Ex + c) : z4;
  float4 ey = in ? ld4(Ey + c) : z4;
  float4 ey_m = jdn ? ld4(Ey + c - sj) : z4;
  // H^{n+1/2} at (j, k0-1): Hx and Hy, recomputed
  float hxp[4] = {0.f, 0.f, 0.f, 0.f}, hyp[4] = {0.f, 0.f, 0.f, 0.f};
  if (p.k0 > 0) {
    const size_t cb = c - sk;
    const float4 hx0 = in ? ld4(Hx + cb) : z4;
    const float4 hy0 = in ? ld4(Hy + cb) : z4;
    const float4 ez0 = in ? ld4(Ez + cb) : z4;
    const float4 ex0 = in ? ld4(Ex + cb) : z4;
    const float4 ey0 = in ? ld4(Ey + cb) : z4;
    const float4 ez0_j = jup ? ld4(Ez + cb + sj) : z4;
    float ez0_e = lane_east_open(ez0.x);
    if (p.lane == 63 && in && p.i0 + 4 < f.P) ez0_e = Ez[cb + 4];
    const int k = p.k0 - 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = p.i0 + e;
      const float eze = e < 3 ? comp(ez0, e + 1) : ez0_e;
      hxp[e] = (i <= N && j < N && k < N)
                   ? comp(hx0, e) - dt * ((comp(ez0_j, e) - comp(ez0, e)) - (comp(ey, e) - comp(ey0, e))) : comp(hx0, e);
      hyp[e] = (i < N && k < N) ? comp(hy0, e) - dt * ((comp(ex, e) - comp(ex0, e)) - (eze - comp(ez0, e))) : comp(hy0, e);
    }
  }
  for (int k = p.k0; k < p.k1; ++k, c += sk) {
    const bool kup = in && k < N;
    const float4 ez = in ? ld4(Ez + c) : z4;
    const float4 hx = in ? ld4(Hx + c) : z4;
    const float4 hy = in ? ld4(Hy + c) : z4;
    const float4 hz = in ? ld4(Hz + c) : z4;
    const float4 ex_k = kup ? ld4(Ex + c + sk) : z4;    // k+1
    const float4 ey_k = kup ? ld4(Ey + c + sk) : z4;
    const float4 ez_j = jup ? ld4(Ez + c + sj) : z4;    // j+1
    const float4 ex_j = jup ? ld4(Ex + c + sj) : z4;
    // the j-1 row: E^n and H^{n-1/2}
    const float4 ex_m = jdn ? ld4(Ex + c - sj) : z4;
    const float4 ez_m = jdn ? ld4(Ez + c - sj) : z4;
    const float4 hx_m = jdn ? ld4(Hx + c - sj) : z4;
    const float4 hz_m = jdn ? ld4(Hz + c - sj) : z4;
    const float4 ey_mk = jdn && k < N ? ld4(Ey + c - sj + sk) : z4;
    // i+4 of Ey, Ez (row j) and Ey (row j-1): next lane, else memory
    float ey_e = lane_east_open(ey.x);
    float ez_e = lane_east_open(ez.x);
    float eym_e = lane_east_open(ey_m.x);
    if (p.lane == 63 && in && p.i0 + 4 < f.P) {
      ey_e = Ey[c + 4];
      ez_e = Ez[c + 4];
      if (jdn) eym_e = Ey[c - sj + 4];
    }
    // H^{n+1/2} at (j, k) (stored) and at (j-1, k) (Hx, Hz, recomputed)
    float hxn[4], hyn[4], hzn[4], hxm[4], hzm[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = p.i0 + e;
      const float eyc = comp(ey, e), ezc = comp(ez, e), exc = comp(ex, e);
      const float eye = e < 3 ? comp(ey, e + 1) : ey_e;
      const float eze = e < 3 ? comp(ez, e + 1) : ez_e;
      hxn[e] = (i <= N && j < N && k < N)
                   ? comp(hx, e) - dt * ((comp(ez_j, e) - ezc) - (comp(ey_k, e) - eyc)) : comp(hx, e);
      hyn[e] = (i < N && k < N) ? comp(hy, e) - dt * ((comp(ex_k, e) - exc) - (eze - ezc)) : comp(hy, e);
      hzn[e] = (i < N && j < N) ? comp(hz, e) - dt * ((eye - eyc) - (comp(ex_j, e) - exc)) : comp(hz, e);
      const float eymc = comp(ey_m, e);
      const float eyme = e < 3 ? comp(ey_m, e + 1) : eym_e;
      hxm[e] = (i <= N && k < N)
                   ? comp(hx_m, e) - dt * ((ezc - comp(ez_m, e)) - (comp(ey_mk, e) - eymc)) : comp(hx_m, e);
      hzm[e] = i < N ? comp(hz_m, e) - dt * ((eyme - eymc) - (exc - comp(ex_m, e))) : comp(hz_m, e);
    }
    if (!jdn) {
#pragma unroll
      for (int e = 0; e < 4; ++e) hxm[e] = hzm[e] = 0.f;
    }
    // H^{n+1/2} at i0-1 (Hz, Hy): previous lane, else recomputed
    float hz_w = lane_west_open(hzn[3]);
    float hy_w = lane_west_open(hyn[3]);
    if (p.lane == 0 && in && p.i0 > 0) {
      const int i = p.i0 - 1;
      const size_t w = c - 1;
      const float eyw = Ey[w], exw = Ex[w], ezw = Ez[w];
      hz_w = (i < N && j < N) ? Hz[w] - dt * ((ey.x - eyw) - (Ex[w + sj] - exw)) : Hz[w];
      hy_w = (i < N && k < N) ? Hy[w] - dt * ((Ex[w + sk] - exw) - (ez.x - ezw)) : Hy[w];
    }
    const bool kk = k >= 1 && k <= N - 1;
    float ox[4], oy[4], oz[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = p.i0 + e;
      const bool ii = i >= 1 && i <= N - 1;
      const float hzw = e > 0 ? hzn[e - 1] : hz_w;
      const float hyw = e > 0 ? hyn[e - 1] : hy_w;
      ox[e] = (i < N && jj && kk) ? comp(ex, e) + dt * ((hzn[e] - hzm[e]) - (hyn[e] - hyp[e])) : comp(ex, e);
      oy[e] = (j < N && ii && kk) ? comp(ey, e) + dt * ((hxn[e] - hxp[e]) - (hzn[e] - hzw)) : comp(ey, e);
      oz[e] = (k < N && ii && jj) ? comp(ez, e) + dt * ((hyn[e] - hyw) - (hxn[e] - hxm[e])) : comp(ez, e);
    }
    if (in) {
      st4o<NT>(oHx + c, hxn[0], hxn[1], hxn[2], hxn[3]);
      st4o<NT>(oHy + c, hyn[0], hyn[1], hyn[2], hyn[3]);
      st4o<NT>(oHz + c, hzn[0], hzn[1], hzn[2], hzn[3]);
      st4o<NT>(oEx + c, ox[0], ox[1], ox[2], ox[3]);
      st4o<NT>(oEy + c, oy[0], oy[1], oy[2], oy[3]);
      st4o<NT>(oEz + c, oz[0], oz[1], oz[2], oz[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      hxp[e] = hxn[e];
      hyp[e] = hyn[e];
    }
    ex = ex_k;
    ey = ey_k;
    ey_m = ey_mk;
  }
}

bool make_fdtd_fused(Launch &L, const FdtdFusedArgs &a, int kc, bool nt) {
  if (kc == 1 && nt) L.set((const void *)fdtd_fused_kernel<1, true>, march_grid<1>(a.N, a.P), dim3(256), 0, a);
  else if (kc == 1) L.set((const void *)fdtd_fused_kernel<1, false>, march_grid<1>(a.N, a.P), dim3(256), 0, a);
  else if (kc == 8) L.set((const void *)fdtd_fused_kernel<8, false>, march_grid<8>(a.N, a.P), dim3(256), 0, a);
  else return false;
  return true;
}

// Soft source (the third kernel of a step): reads the device step counter n,
// adds g[n] to Ez at the source node, records the probe, increments n.  The
// counter lives on the device so a replayed graph sees the absolute step.
// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking, variant 8 with depth 2).
//
// A block owns an output tile of 60 nodes along i x 13 rows along j x tk
// planes along k and marches through its planes.  Lane l of wave w holds
// node (i0 - 2 + l, j0 - 2 + w): each step's H update needs E at i+1, j+1,
// k+1 and its E update H at i-1, j-1, k-1, so two steps need two nodes /
// rows of halo below the tile and one above; halo nodes are recomputed by
// the neighbouring blocks as well (60 of 64 lanes and 13 of 16 rows are
// outputs).  Along i the neighbour is the adjacent lane (DPP); along j the
// rows of the intermediate fields that other waves need pass through LDS;
// along k a thread keeps the previous plane of each field in registers.
// Iteration m of the march computes, for the wave's row:
//   A  H^{n+1/2} of plane m      (E^n of planes m, m+1; rows j, j+1)
//   B  E^{n+1}   of plane m      (+ the source of step n), from H^{n+1/2}
//                                of planes m-1, m and rows j-1, j
//   C  H^{n+3/2} of plane m-1    from E^{n+1} of planes m-1, m, rows j, j+1
//   D  E^{n+2}   of plane m-1    (+ the source of step n+1), from H^{n+3/2}
//                                of planes m-2, m-1 and rows j-1, j
// and stores plane m-1 of the outputs.  Two barriers per plane: after A
// (B reads row j-1 of H^{n+1/2}) and after C (D reads row j-1 of
// H^{n+3/2}); C reads row j+1 of E^{n+1} of plane m-1, written in the
// previous iteration (double-buffered by plane parity).  Every update is the
// one-step kernels' expression with the same operand order, and a node that
// a step does not update keeps its value, so two launches of the fused step
// and one launch of this kernel give the same bits.
// ---------------------------------------------------------------------------
constexpr int kTbNW = 16;              // waves (rows) per block
constexpr int kTbTJ = kTbNW - 3;       // output rows per block
constexpr int kTbTI = 60;              // output nodes along i per block

template <bool NT>
__device__ __forceinline__ void st1(float *p, float v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <bool NT>
__global__ __launch_bounds__(1024) void fdtd_tb2_kernel(const FdtdTbArgs a) {
  __shared__ float sH1[2][kTbNW][64];      // H^{n+1/2} x, z of the current plane
  __shared__ float sE1[2][2][kTbNW][64];   // [plane parity][x, z] E^{n+1}
  __shared__ float sH2[2][kTbNW][64];      // H^{n+3/2} x, z
  const int nb = a.ni * a.nj * a.nk;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;                    // the whole block: before any barrier
  const int ti = lb % a.ni, tj = (lb / a.ni) % a.nj, tkk = lb / (a.ni * a.nj);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int N = a.N, M = N + 1;
  const int i = ti * kTbTI - 2 + lane;
  const int j = tj * kTbTJ - 2 + w;
  const int kb = tkk * a.tk, ke = min(kb + a.tk, M);   // output planes [kb, ke)
  const bool iv = i >= 0 && i <= N, jv = j >= 0 && j <= N, vld = iv && jv;
  const bool jup = vld && j + 1 <= N;
  const bool out_ij = vld && lane >= 2 && lane < 2 + kTbTI && w >= 2 && w < 2 + kTbTJ;
  const bool ii = i >= 1 && i <= N - 1, jj = j >= 1 && j <= N - 1;
  const bool ilt = i < N, jlt = j < N;
  const int wm = w > 0 ? w - 1 : 0, wp = w < kTbNW - 1 ? w + 1 : kTbNW - 1;
  const size_t sk = (size_t)M * a.P;
  const size_t cij = vld ? (size_t)j * a.P + i : 0;
  const float dt = a.dt;
  const long long n = *a.step;
  const bool add0 = n >= 0 && n < a.glen, add1 = n + 1 >= 0 && n + 1 < a.glen;
  const float g0 = add0 ? a.g[n] : 0.f, g1 = add1 ? a.g[n + 1] : 0.f;
  const bool srcij = i == a.si && j == a.sj;

  auto ld = [&](const float *f, int k, bool ok) -> float { return ok && k >= 0 && k <= N ? f[k * sk + cij] : 0.f; };
  auto ldj = [&](const float *f, int k) -> float {           // row j+1
    return jup && k >= 0 && k <= N ? f[k * sk + cij + a.P] : 0.f;
  };

  const int m0 = max(kb - 2, 0);
  // E^n of plane m0 (own row)
  float ex = ld(a.Ex, m0, vld), ey = ld(a.Ey, m0, vld), ez = ld(a.Ez, m0, vld);
  float h1x_p = 0.f, h1y_p = 0.f, h1z_p = 0.f;      // H^{n+1/2} of plane m-1
  float e1x_p = 0.f, e1y_p = 0.f, e1z_p = 0.f;      // E^{n+1} of plane m-1
  float h2x_p = 0.f, h2y_p = 0.f;                   // H^{n+3/2} of plane m-2
  // loads one plane ahead: E^n of plane m+1, row j+1 of E^n and H of plane m
  float exk = ld(a.Ex, m0 + 1, vld), eyk = ld(a.Ey, m0 + 1, vld), ezk = ld(a.Ez, m0 + 1, vld);
  float ex_j = ldj(a.Ex, m0), ez_j = ldj(a.Ez, m0);
  float hx = ld(a.Hx, m0, vld), hy = ld(a.Hy, m0, vld), hz = ld(a.Hz, m0, vld);
  for (int m = m0; m <= ke; ++m) {
    const bool pm = m <= N;                          // plane m exists
    // the next iteration's operands, in flight during this one
    const float nexk = ld(a.Ex, m + 2, vld), neyk = ld(a.Ey, m + 2, vld), nezk = ld(a.Ez, m + 2, vld);
    const float nex_j = ldj(a.Ex, m + 1), nez_j = ldj(a.Ez, m + 1);
    const float nhx = ld(a.Hx, m + 1, vld), nhy = ld(a.Hy, m + 1, vld), nhz = ld(a.Hz, m + 1, vld);
    // ---- A: H^{n+1/2} of plane m
    const float ey_e = lane_east_open(ey), ez_e = lane_east_open(ez);
    const bool mlt = m < N;
    const float h1x = (jlt && mlt) ? hx - dt * ((ez_j - ez) - (eyk - ey)) : hx;
    const float h1y = (ilt && mlt) ? hy - dt * ((exk - ex) - (ez_e - ez)) : hy;
    const float h1z = (ilt && jlt) ? hz - dt * ((ey_e - ey) - (ex_j - ex)) : hz;
    sH1[0][w][lane] = h1x;
    sH1[1][w][lane] = h1z;
    __syncthreads();
    // ---- B: E^{n+1} of plane m
    const float h1x_jm = sH1[0][wm][lane], h1z_jm = sH1[1][wm][lane];
    const float h1z_w = lane_west_open(h1z), h1y_w = lane_west_open(h1y);
    const bool kk = m >= 1 && m <= N - 1;
    const float e1x = (ilt && jj && kk) ? ex + dt * ((h1z - h1z_jm) - (h1y - h1y_p)) : ex;
    const float e1y = (jlt && ii && kk) ? ey + dt * ((h1x - h1x_p) - (h1z - h1z_w)) : ey;
    float e1z = (mlt && ii && jj) ? ez + dt * ((h1y - h1y_w) - (h1x - h1x_jm)) : ez;
    if (srcij && m == a.sk) {
      if (add0) e1z = e1z + g0;
      if (out_ij && m >= kb && m < ke && n >= 0 && n < a.pcap) a.probe[n] = e1z;
    }
    sE1[m & 1][0][w][lane] = pm ? e1x : 0.f;
    sE1[m & 1][1][w][lane] = pm ? e1z : 0.f;
    // ---- C: H^{n+3/2} of plane q = m-1 (E^{n+1} of row j+1, plane q, from
    // the previous iteration's buffer)
    const int q = m - 1;
    const bool doC = q >= 0 && q >= kb - 1 && q <= ke - 1;
    float h2x = 0.f, h2y = 0.f, h2z = 0.f;
    if (doC) {
      const float e1x_jq = sE1[q & 1][0][wp][lane], e1z_jq = sE1[q & 1][1][wp][lane];
      const float e1xn = pm ? e1x : 0.f, e1yn = pm ? e1y : 0.f;   // E^{n+1} of plane q+1
      // the i+1 neighbours, taken on every lane before the selects below
      // (inside a select arm only the lanes of that arm would run the lane
      // shift, and the lane before one of the others would read 0)
      const float e1z_e = lane_east_open(e1z_p), e1y_e = lane_east_open(e1y_p);
      const bool qlt = q < N;
      h2x = (jlt && qlt) ? h1x_p - dt * ((e1z_jq - e1z_p) - (e1yn - e1y_p)) : h1x_p;
      h2y = (ilt && qlt) ? h1y_p - dt * ((e1xn - e1x_p) - (e1z_e - e1z_p)) : h1y_p;
      h2z = (ilt && jlt) ? h1z_p - dt * ((e1y_e - e1y_p) - (e1x_jq - e1x_p)) : h1z_p;
    }
    sH2[0][w][lane] = h2x;
    sH2[1][w][lane] = h2z;
    __syncthreads();
    // ---- D: E^{n+2} of plane q, and the outputs of plane q
    if (q >= kb && q <= ke - 1) {
      const float h2x_jm = sH2[0][wm][lane], h2z_jm = sH2[1][wm][lane];
      const float h2z_w = lane_west_open(h2z), h2y_w = lane_west_open(h2y);
      const bool kq = q >= 1 && q <= N - 1;
      const float e2x = (ilt && jj && kq) ? e1x_p + dt * ((h2z - h2z_jm) - (h2y - h2y_p)) : e1x_p;
      const float e2y = (jlt && ii && kq) ? e1y_p + dt * ((h2x - h2x_p) - (h2z - h2z_w)) : e1y_p;
      float e2z = (q < N && ii && jj) ? e1z_p + dt * ((h2y - h2y_w) - (h2x - h2x_jm)) : e1z_p;
      if (srcij && q == a.sk) {
        if (add1) e2z = e2z + g1;
        if (out_ij && n + 1 >= 0 && n + 1 < a.pcap) a.probe[n + 1] = e2z;
      }
      if (out_ij) {
        const size_t c = (size_t)q * sk + cij;
        st1<NT>(a.oEx + c, e2x);
        st1<NT>(a.oEy + c, e2y);
        st1<NT>(a.oEz + c, e2z);
        st1<NT>(a.oHx + c, h2x);
        st1<NT>(a.oHy + c, h2y);
        st1<NT>(a.oHz + c, h2z);
      }
    }
    // ---- rotate: plane m becomes the previous plane
    h2x_p = h2x;
    h2y_p = h2y;
    h1x_p = h1x;
    h1y_p = h1y;
    h1z_p = h1z;
    e1x_p = e1x;
    e1y_p = e1y;
    e1z_p = e1z;
    ex = exk;
    ey = eyk;
    ez = ezk;
    exk = nexk;
    eyk = neyk;
    ezk = nezk;
    ex_j = nex_j;
    ez_j = nez_j;
    hx = nhx;
    hy = nhy;
    hz = nhz;
  }
}

bool make_fdtd_tb2(Launch &L, const FdtdTbArgs &a0, bool nt) {
  FdtdTbArgs a = a0;
  const int M = a.N + 1;
  a.ni = (M + kTbTI - 1) / kTbTI;
  a.nj = (M + kTbTJ - 1) / kTbTJ;
  // plane segments of equal length, as many as fill the chip in one round
  // (two blocks of 16 waves per compute unit), at least 8 planes each
  const int slots = 2 * kCUs;
  a.nk = std::max(1, std::min((slots + a.ni * a.nj / 2) / (a.ni * a.nj), M / 8));
  a.tk = (M + a.nk - 1) / a.nk;
  a.nk = (M + a.tk - 1) / a.tk;
  const int nb = a.ni * a.nj * a.nk;
  const dim3 grid((unsigned)xcd_padded_grid(nb));
  if (nt) L.set((const void *)fdtd_tb2_kernel<true>, grid, dim3(64 * kTbNW), 0, a);
  else L.set((const void *)fdtd_tb2_kernel<false>, grid, dim3(64 * kTbNW), 0, a);
  return true;
}

// ---------------------------------------------------------------------------
// Two steps per launch over whole rows (variants 9 and 10 with depth 2,
// N <= 256).
//
// The scheme of the kernel above (blocks march along k; phases A-D per
// plane, two barriers; rows j-1 / j+1 of the intermediate fields through
// LDS; two rows below and one above the output rows recomputed) with a
// wave holding a whole row: lane l keeps nodes 4l .. 4l+3, read and written
// as 16-byte vectors, so no node along i is computed twice and a wave issues
// a quarter of the memory instructions.  A node's i+1 neighbour is the next
// element of the lane, or element 0 of the next lane (lane shift); its i-1
// neighbour likewise.  Elements past N (row padding) take no update and
// keep their values.
//
// At N = 256 a row has 257 nodes and lane 63 ends at i = 255.  The node at
// i = N takes part only through its E values, the i+1 neighbours of node
// N-1: no E component at i = N is ever updated (Ex there is row padding, Ey
// and Ez are tangential to the wall), so E^{n+1} = E^n there and lane 63
// reads them from the input set.  Nor do Hy and Hz there change, and the
// library keeps the column's E, Hy and Hz equal in both field sets (every
// kernel that writes a whole set copies them, kb_write mirrors them), so of
// the column only Hx is written: lane 63 updates it twice with the
// column's unchanging E (E_z of row j+1 from the next wave through LDS).
//
// The block that finishes last (a counter of finished blocks, reset by
// that block) advances the device step counter by the launch's two steps:
// every other block has read it by then.
// ---------------------------------------------------------------------------

struct Q4 {
  float v[4];
};
// Plane accesses through buffer resources: the plane's address and byte
// size in scalar registers, a lane's 32-bit byte offset in a vector
// register.  The hardware range check does the domain masking: a load
// outside the plane (offset kOff, or a plane of size 0 for k outside
// 0..N) returns zero and a store there is dropped.  So every path issues
// the same memory instructions (a wait for an earlier load then need not
// wait for all), no lane keeps a 64-bit address, and no zero has to be
// written into the destination first.
typedef float V4f __attribute__((ext_vector_type(4)));
typedef unsigned V4u __attribute__((ext_vector_type(4)));   // the buffer builtins' data type
constexpr unsigned kOff = 0x80000000u;        // an offset beyond every plane
constexpr int kRsrcWord3 = 0x00020000;        // raw buffer, 32-bit data (gfx9 family)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *plane, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(plane), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ Q4 q4ld(__amdgpu_buffer_rsrc_t r, unsigned ob) {
  const V4f a = __builtin_bit_cast(V4f, __builtin_amdgcn_raw_buffer_load_b128(r, ob, 0, 0));
  return Q4{{a.x, a.y, a.z, a.w}};
}
__device__ __forceinline__ float f1ld(__amdgpu_buffer_rsrc_t r, unsigned ob) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, ob, 0, 0));
}
__device__ __forceinline__ void f1st(__amdgpu_buffer_rsrc_t r, unsigned ob, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, ob, 0, 0);
}
// NT: non-temporal (streaming) store
template <bool NT>
__device__ __forceinline__ void q4st(__amdgpu_buffer_rsrc_t r, unsigned ob, const Q4 &a) {
  const V4f v = {a.v[0], a.v[1], a.v[2], a.v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4u, v), r, ob, 0, NT ? 2 : 0);
}
__device__ __forceinline__ float4 f4of(const Q4 &a) { return make_float4(a.v[0], a.v[1], a.v[2], a.v[3]); }
__device__ __forceinline__ Q4 q4of(const float4 &a) { return Q4{{a.x, a.y, a.z, a.w}}; }
// i+1 and i-1 neighbours of the lane's four nodes (whole-wave lane shifts:
// call from code every lane of the wave runs)
__device__ __forceinline__ Q4 q4east(const Q4 &a, bool last, float ext) {
  float t = lane_east_open(a.v[0]);
  if (last) t = ext;
  return Q4{{a.v[1], a.v[2], a.v[3], t}};
}
__device__ __forceinline__ Q4 q4west(const Q4 &a) {
  return Q4{{lane_west_open(a.v[3]), a.v[0], a.v[1], a.v[2]}};
}

// NW waves (rows) per block, NW - 3 output rows; PF: operands loaded one
// plane ahead (the register room for it needs NW <= 12); FR: N = 256, every
// lane's four nodes lie in the row (the per-node conditions fold away)
template <bool NT, int NW, bool PF, bool FR>
__global__ __launch_bounds__(64 * NW) void fdtd_tb2_rows_kernel(const FdtdTbArgs a) {
  constexpr int kTrNW = NW, kTrTJ = NW - 3;
  __shared__ float4 sH1[2][kTrNW][64];      // H^{n+1/2} x, z of the current plane
  __shared__ float4 sE1[2][2][kTrNW][64];   // [plane parity][x, z] E^{n+1}
  __shared__ float4 sH2[2][kTrNW][64];      // H^{n+3/2} x, z
  __shared__ float sEzN[kTrNW];             // E_z at i = N of each row, current plane
  const int nb = a.nj * a.nk;
  const int lb = xcd_logical_block(nb);
  // the last block of the grid to finish advances the step counter (no
  // fence: the block's read of the counter has returned before this)
  auto finish = [&]() {
    if (threadIdx.x == 0) {
      if (atomicAdd(a.done, 1u) == gridDim.x - 1) {
        atomicExch(a.done, 0u);
        *a.step_w += 2;
      }
    }
  };
  if (lb >= nb) {                           // the whole block: before any barrier
    finish();
    return;
  }
  const int tj = lb % a.nj, tkk = lb / a.nj;
  // w is the same in the whole wave: read once, so that everything that
  // depends on the row only sits in scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int N = a.N, M = N + 1;
  const int i0 = 4 * lane;
  const int j = tj * kTrTJ - 2 + w;
  const int kb = tkk * a.tk, ke = min(kb + a.tk, M);   // output planes [kb, ke)
  const bool jv = j >= 0 && j <= N;
  const bool vld = jv && (FR || i0 <= N);              // the lane holds a node of the row
  const bool jup = vld && j + 1 <= N;
  const bool out = vld && w >= 2 && w < 2 + kTrTJ;
  const bool jj = j >= 1 && j <= N - 1, jlt = j < N;
  const bool last = lane == 63;
  const bool xn = FR && last && jv;                     // lane 63 reads E at i = N
  // per-node conditions, evaluated where used (kept as lane masks they
  // would tie up scalar registers the kernel needs)
  auto iN = [&](int e) { return FR || i0 + e <= N; };
  auto ilt = [&](int e) { return FR || i0 + e < N; };
  auto ii = [&](int e) { return FR ? (e > 0 || lane > 0) : (i0 + e >= 1) & (i0 + e <= N - 1); };
  const bool srow = j == a.sj && a.si >= i0 && a.si < i0 + 4;   // the source node is in this lane
  const int wm = w > 0 ? w - 1 : 0, wp = w < kTrNW - 1 ? w + 1 : kTrNW - 1;
  const size_t sk = (size_t)M * a.P;
  // byte offsets within a plane (a plane has at most 257 x 260 floats);
  // kOff where the lane has no such node
  const unsigned pbytes = (unsigned)(M * a.P * 4);
  const unsigned ob = vld ? (unsigned)((j * a.P + i0) * 4) : kOff;
  const unsigned obj = jup ? (unsigned)(((j + 1) * a.P + i0) * 4) : kOff;
  const unsigned obN = xn ? (unsigned)((j * a.P + N) * 4) : kOff;
  auto plane = [&](const float *f, int k) {   // plane k of a field (size 0 outside 0..N)
    return plane_rsrc(f + (size_t)k * sk, k >= 0 && k <= N ? pbytes : 0u);
  };
  const float dt = a.dt;
  const long long n = *a.step;
  const bool add0 = n >= 0 && n < a.glen, add1 = n + 1 >= 0 && n + 1 < a.glen;
  const float g0 = add0 ? a.g[n] : 0.f, g1 = add1 ? a.g[n + 1] : 0.f;
  const Q4 z4{{0.f, 0.f, 0.f, 0.f}};

  // operands outside the domain read as zero
  auto ld = [&](const float *f, int k) -> Q4 { return q4ld(plane(f, k), ob); };
  auto ldj = [&](const float *f, int k) -> Q4 { return q4ld(plane(f, k), obj); };   // row j+1
  auto ldN = [&](const float *f, int k) -> float { return f1ld(plane(f, k), obN); };

  const int m0 = max(kb - 2, 0);
  Q4 ex = ld(a.Ex, m0), ey = ld(a.Ey, m0), ez = ld(a.Ez, m0);   // E^n of plane m
  float eyN = ldN(a.Ey, m0), ezN = ldN(a.Ez, m0);               // E at i = N, plane m
  float eyN_p = 0.f, ezN_p = 0.f;                               // ... plane m-1
  Q4 h1x_p = z4, h1y_p = z4, h1z_p = z4;       // H^{n+1/2} of plane m-1
  Q4 e1x_p = z4, e1y_p = z4, e1z_p = z4;       // E^{n+1} of plane m-1
  Q4 h2x_p = z4, h2y_p = z4;                   // H^{n+3/2} of plane m-2
  // with PF: E^n of plane m+1, row j+1 of E^n and H of plane m are loaded
  // one iteration ahead
  Q4 pexk = z4, peyk = z4, pezk = z4, pex_j = z4, pez_j = z4, phx = z4, phy = z4, phz = z4;
  float peyNk = 0.f, pezNk = 0.f, phxN = 0.f;
  if constexpr (PF) {
    pexk = ld(a.Ex, m0 + 1); peyk = ld(a.Ey, m0 + 1); pezk = ld(a.Ez, m0 + 1);
    pex_j = ldj(a.Ex, m0); pez_j = ldj(a.Ez, m0);
    phx = ld(a.Hx, m0); phy = ld(a.Hy, m0); phz = ld(a.Hz, m0);
    peyNk = ldN(a.Ey, m0 + 1); pezNk = ldN(a.Ez, m0 + 1); phxN = ldN(a.Hx, m0);
  }
  for (int m = m0; m <= ke; ++m) {
    const bool pm = m <= N;                          // plane m exists
    Q4 exk, eyk, ezk, ex_j, ez_j, hx, hy, hz;
    float eyNk, ezNk, hxN;                           // hxN: Hx at i = N (lane 63 at N = 256)
    if constexpr (PF) {
      exk = pexk; eyk = peyk; ezk = pezk; ex_j = pex_j; ez_j = pez_j; hx = phx; hy = phy; hz = phz;
      eyNk = peyNk; ezNk = pezNk; hxN = phxN;
      pexk = ld(a.Ex, m + 2); peyk = ld(a.Ey, m + 2); pezk = ld(a.Ez, m + 2);
      pex_j = ldj(a.Ex, m + 1); pez_j = ldj(a.Ez, m + 1);
      phx = ld(a.Hx, m + 1); phy = ld(a.Hy, m + 1); phz = ld(a.Hz, m + 1);
      peyNk = ldN(a.Ey, m + 2); pezNk = ldN(a.Ez, m + 2); phxN = ldN(a.Hx, m + 1);
    } else {
      exk = ld(a.Ex, m + 1); eyk = ld(a.Ey, m + 1); ezk = ld(a.Ez, m + 1);
      ex_j = ldj(a.Ex, m); ez_j = ldj(a.Ez, m);
      hx = ld(a.Hx, m); hy = ld(a.Hy, m); hz = ld(a.Hz, m);
      eyNk = ldN(a.Ey, m + 1); ezNk = ldN(a.Ez, m + 1); hxN = ldN(a.Hx, m);
    }
    // ---- A: H^{n+1/2} of plane m
    const bool mlt = m < N;
    const Q4 ey_e = q4east(ey, last, eyN), ez_e = q4east(ez, last, ezN);
    Q4 h1x, h1y, h1z;
    // (every update is computed and then selected, its condition combined
    // without short-circuits: a conditional expression would become a
    // branch per node and component)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float ux = hx.v[e] - dt * ((ez_j.v[e] - ez.v[e]) - (eyk.v[e] - ey.v[e]));
      const float uy = hy.v[e] - dt * ((exk.v[e] - ex.v[e]) - (ez_e.v[e] - ez.v[e]));
      const float uz = hz.v[e] - dt * ((ey_e.v[e] - ey.v[e]) - (ex_j.v[e] - ex.v[e]));
      h1x.v[e] = (iN(e) & jlt & mlt) ? ux : hx.v[e];
      h1y.v[e] = (ilt(e) & mlt) ? uy : hy.v[e];
      h1z.v[e] = (ilt(e) & jlt) ? uz : hz.v[e];
    }
    sH1[0][w][lane] = f4of(h1x);
    sH1[1][w][lane] = f4of(h1z);
    if (last) sEzN[w] = ezN;
    __syncthreads();
    // Hx at i = N of plane m (two updates with the same E; the rows j = N
    // and the plane k = N keep it)
    {
      const float d = (sEzN[wp] - ezN) - (eyNk - eyN);
      const float h1 = hxN - dt * d;
      const float h = (jlt & mlt) ? h1 - dt * d : hxN;
      // (only lane 63 of an output row, and planes kb .. ke-1, write)
      const unsigned o = out && m >= kb && m < ke ? obN : kOff;
      f1st(plane(a.oHx, m), o, h);
    }
    // ---- B: E^{n+1} of plane m
    const Q4 h1x_jm = q4of(sH1[0][wm][lane]), h1z_jm = q4of(sH1[1][wm][lane]);
    const Q4 h1z_w = q4west(h1z), h1y_w = q4west(h1y);
    const bool kk = m >= 1 && m <= N - 1;
    Q4 e1x, e1y, e1z;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float ux = ex.v[e] + dt * ((h1z.v[e] - h1z_jm.v[e]) - (h1y.v[e] - h1y_p.v[e]));
      const float uy = ey.v[e] + dt * ((h1x.v[e] - h1x_p.v[e]) - (h1z.v[e] - h1z_w.v[e]));
      const float uz = ez.v[e] + dt * ((h1y.v[e] - h1y_w.v[e]) - (h1x.v[e] - h1x_jm.v[e]));
      e1x.v[e] = (ilt(e) & jj & kk) ? ux : ex.v[e];
      e1y.v[e] = (jlt & ii(e) & kk) ? uy : ey.v[e];
      e1z.v[e] = (mlt & ii(e) & jj) ? uz : ez.v[e];
    }
    if (m == a.sk) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (srow && i0 + e == a.si) {
          if (add0) e1z.v[e] = e1z.v[e] + g0;
          if (out && m >= kb && m < ke && n >= 0 && n < a.pcap) a.probe[n] = e1z.v[e];
        }
    }
    sE1[m & 1][0][w][lane] = pm ? f4of(e1x) : make_float4(0.f, 0.f, 0.f, 0.f);
    sE1[m & 1][1][w][lane] = pm ? f4of(e1z) : make_float4(0.f, 0.f, 0.f, 0.f);
    // ---- C: H^{n+3/2} of plane q = m-1 (E^{n+1} of row j+1, plane q, from
    // the previous iteration's buffer)
    const int q = m - 1;
    const bool doC = q >= 0 && q >= kb - 1 && q <= ke - 1;
    Q4 h2x = z4, h2y = z4, h2z = z4;
    if (doC) {
      const Q4 e1x_jq = q4of(sE1[q & 1][0][wp][lane]), e1z_jq = q4of(sE1[q & 1][1][wp][lane]);
      const Q4 e1xn = pm ? e1x : z4, e1yn = pm ? e1y : z4;   // E^{n+1} of plane q+1
      // i+1 neighbours (at i = N: E^{n+1} = E^n of plane q)
      const Q4 e1z_e = q4east(e1z_p, last, ezN_p), e1y_e = q4east(e1y_p, last, eyN_p);
      const bool qlt = q < N;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float ux = h1x_p.v[e] - dt * ((e1z_jq.v[e] - e1z_p.v[e]) - (e1yn.v[e] - e1y_p.v[e]));
        const float uy = h1y_p.v[e] - dt * ((e1xn.v[e] - e1x_p.v[e]) - (e1z_e.v[e] - e1z_p.v[e]));
        const float uz = h1z_p.v[e] - dt * ((e1y_e.v[e] - e1y_p.v[e]) - (e1x_jq.v[e] - e1x_p.v[e]));
        h2x.v[e] = (iN(e) & jlt & qlt) ? ux : h1x_p.v[e];
        h2y.v[e] = (ilt(e) & qlt) ? uy : h1y_p.v[e];
        h2z.v[e] = (ilt(e) & jlt) ? uz : h1z_p.v[e];
      }
    }
    sH2[0][w][lane] = f4of(h2x);
    sH2[1][w][lane] = f4of(h2z);
    __syncthreads();
    // ---- D: E^{n+2} of plane q, and the outputs of plane q
    if (q >= kb && q <= ke - 1) {
      const Q4 h2x_jm = q4of(sH2[0][wm][lane]), h2z_jm = q4of(sH2[1][wm][lane]);
      const Q4 h2z_w = q4west(h2z), h2y_w = q4west(h2y);
      const bool kq = q >= 1 && q <= N - 1;
      Q4 e2x, e2y, e2z;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float ux = e1x_p.v[e] + dt * ((h2z.v[e] - h2z_jm.v[e]) - (h2y.v[e] - h2y_p.v[e]));
        const float uy = e1y_p.v[e] + dt * ((h2x.v[e] - h2x_p.v[e]) - (h2z.v[e] - h2z_w.v[e]));
        const float uz = e1z_p.v[e] + dt * ((h2y.v[e] - h2y_w.v[e]) - (h2x.v[e] - h2x_jm.v[e]));
        e2x.v[e] = (ilt(e) & jj & kq) ? ux : e1x_p.v[e];
        e2y.v[e] = (jlt & ii(e) & kq) ? uy : e1y_p.v[e];
        e2z.v[e] = ((q < N) & ii(e) & jj) ? uz : e1z_p.v[e];
      }
      if (q == a.sk) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (srow && i0 + e == a.si) {
            if (add1) e2z.v[e] = e2z.v[e] + g1;
            if (out && n + 1 >= 0 && n + 1 < a.pcap) a.probe[n + 1] = e2z.v[e];
          }
      }
      const unsigned o = out ? ob : kOff;
      q4st<NT>(plane(a.oEx, q), o, e2x);
      q4st<NT>(plane(a.oEy, q), o, e2y);
      q4st<NT>(plane(a.oEz, q), o, e2z);
      q4st<NT>(plane(a.oHx, q), o, h2x);
      q4st<NT>(plane(a.oHy, q), o, h2y);
      q4st<NT>(plane(a.oHz, q), o, h2z);
    }
    // ---- rotate: plane m becomes the previous plane
    h2x_p = h2x;
    h2y_p = h2y;
    h1x_p = h1x;
    h1y_p = h1y;
    h1z_p = h1z;
    e1x_p = e1x;
    e1y_p = e1y;
    e1z_p = e1z;
    ex = exk;
    ey = eyk;
    ez = ezk;
    eyN_p = eyN;
    ezN_p = ezN;
    eyN = eyNk;
    ezN = ezNk;
  }
  finish();
}

bool make_fdtd_tb2_rows(Launch &L, const FdtdTbArgs &a0, bool nt, int form) {
  FdtdTbArgs a = a0;
  const int M = a.N + 1;
  if (a.N > 4 * 64 || a.P % 4 != 0) return false;
  // form 0: 16 waves per block, operands loaded in the iteration that uses
  // them; form 1: 12 waves, loaded one plane ahead
  const int nw = form == 0 ? 16 : 12;
  a.ni = 1;
  a.nj = (M + nw - 4) / (nw - 3);
  // plane segments of equal length, as many as fill the chip with one
  // block (up to 128 KiB of LDS) per compute unit, at least 8 planes each
  a.nk = std::max(1, std::min(kCUs / a.nj, M / 8));
  a.tk = (M + a.nk - 1) / a.nk;
  a.nk = (M + a.tk - 1) / a.tk;
  const int nb = a.nj * a.nk;
  const dim3 grid((unsigned)xcd_padded_grid(nb));
  const bool fr = a.N == 4 * 64;
  const void *f = form == 0
      ? (fr ? (nt ? (const void *)fdtd_tb2_rows_kernel<true, 16, false, true>
                  : (const void *)fdtd_tb2_rows_kernel<false, 16, false, true>)
            : (nt ? (const void *)fdtd_tb2_rows_kernel<true, 16, false, false>
                  : (const void *)fdtd_tb2_rows_kernel<false, 16, false, false>))
      : (fr ? (nt ? (const void *)fdtd_tb2_rows_kernel<true, 12, true, true>
                  : (const void *)fdtd_tb2_rows_kernel<false, 12, true, true>)
            : (nt ? (const void *)fdtd_tb2_rows_kernel<true, 12, true, false>
                  : (const void *)fdtd_tb2_rows_kernel<false, 12, true, false>));
  L.set(f, grid, dim3(64 * nw), 0, a);
  return true;
}

// Two nodes per lane (rows of up to 129 nodes fill the wave): the same
// accesses and lane shifts as Q4 with 8-byte loads, stores and LDS slots.
struct Q2 {
  float v[2];
};
typedef float V2f __attribute__((ext_vector_type(2)));
typedef unsigned V2u __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Q2 qeast(const Q2 &a, bool last, float ext) {
  float t = lane_east_open(a.v[0]);
  if (last) t = ext;
  return Q2{{a.v[1], t}};
}
__device__ __forceinline__ Q2 qwest(const Q2 &a) { return Q2{{lane_west_open(a.v[1]), a.v[0]}}; }
__device__ __forceinline__ Q4 qeast(const Q4 &a, bool last, float ext) { return q4east(a, last, ext); }
__device__ __forceinline__ Q4 qwest(const Q4 &a) { return q4west(a); }
__device__ __forceinline__ float2 ldsof(const Q2 &a) { return make_float2(a.v[0], a.v[1]); }
__device__ __forceinline__ float4 ldsof(const Q4 &a) { return f4of(a); }
__device__ __forceinline__ Q2 qof(const float2 &a) { return Q2{{a.x, a.y}}; }
__device__ __forceinline__ Q4 qof(const float4 &a) { return q4of(a); }
template <int NPL> struct QT;
template <> struct QT<4> { typedef Q4 type; typedef float4 lds; };
template <> struct QT<2> { typedef Q2 type; typedef float2 lds; };

// ---------------------------------------------------------------------------
// Three steps per launch over whole rows (variants 9 and 10 with depth 3,
// N <= 256).  The two-step kernel's march with a third pair of phases: per
// plane m, A H^{n+1/2}(m), B E^{n+1}(m), C H^{n+3/2}(m-1), D E^{n+2}(m-1),
// E H^{n+5/2}(m-2), F E^{n+3}(m-2) and the outputs of plane m-2, with a
// barrier after A, C and E.  Rows j-1 of each new H and j+1 of each new E
// pass through LDS; a new E row is written after the barrier that follows
// the reads of the previous plane's row, so each array holds one plane.
// Three rows below and two above the output rows, and three planes below
// each segment, are recomputed: 12 waves (rows) give 7 output rows.  A
// recomputed row runs only the phases whose results an output row depends
// on (rows w in [3, 10) output; F needs E on [2, 10), which needs D on
// [2, 11), C on [1, 11), B on [1, 12) and A everywhere), so the outermost
// rows skip the later phases and their LDS writes.  Each
// layer of the march reads and writes what the two-step kernel's does, for
// three steps instead of two.  The i = N column's Hx (N = 256) takes its
// three updates in lane 63; the last block advances the step counter by 3.
// ---------------------------------------------------------------------------
// Accesses to a plane of all six fields of a set through one buffer
// resource: the fields lie fs bytes apart, so the field's start is the
// instruction's scalar offset (f * fs) and the lane's offset in the plane is
// the vector offset; the resource spans the six planes.  A lane without a
// node (offset kOff) or a plane outside 0..N (size 0) reads zero and drops
// its stores, whether or not the scalar offset enters the range check.
__device__ __forceinline__ Q4 q4ld_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo) {
  const V4f a = __builtin_bit_cast(V4f, __builtin_amdgcn_raw_buffer_load_b128(r, ob, fo, 0));
  return Q4{{a.x, a.y, a.z, a.w}};
}
__device__ __forceinline__ float f1ld_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, ob, fo, 0));
}
__device__ __forceinline__ void f1st_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, ob, fo, 0);
}
template <bool NT>
__device__ __forceinline__ void q4st_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo, const Q4 &a) {
  const V4f v = {a.v[0], a.v[1], a.v[2], a.v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4u, v), r, ob, fo, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void qst_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo, const Q4 &a) {
  q4st_f<NT>(r, ob, fo, a);
}
template <bool NT>
__device__ __forceinline__ void qst_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo, const Q2 &a) {
  const V2f v = {a.v[0], a.v[1]};
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2u, v), r, ob, fo, NT ? 2 : 0);
}
template <int NPL>
__device__ __forceinline__ typename QT<NPL>::type qld_f(__amdgpu_buffer_rsrc_t r, unsigned ob, int fo) {
  if constexpr (NPL == 4) {
    return q4ld_f(r, ob, fo);
  } else {
    const V2f a = __builtin_bit_cast(V2f, __builtin_amdgcn_raw_buffer_load_b64(r, ob, fo, 0));
    return Q2{{a.x, a.y}};
  }
}

// NPL nodes per lane: 4 (rows up to 257 nodes), 2 (up to 129); FR: the row
// is exactly 64 * NPL + 1 nodes (the per-node conditions fold away)
template <bool NT, bool FR, int NPL>
__global__ __launch_bounds__(768) void fdtd_tb3_rows_kernel(const FdtdTbArgs a) {
  constexpr int kNW = 12, kTJ = kNW - 5;
  typedef typename QT<NPL>::type Q;            // a lane's NPL nodes of a row
  typedef typename QT<NPL>::lds LT;
  __shared__ LT sH1[2][kNW][64];   // H^{n+1/2} x, z of plane m
  __shared__ LT sE1[2][kNW][64];   // E^{n+1} x, z of plane m-1 (until C), then m
  __shared__ LT sH2[2][kNW][64];   // H^{n+3/2} x, z of plane m-1
  __shared__ LT sE2[2][kNW][64];   // E^{n+2} x, z of plane m-2 (until E), then m-1
  __shared__ LT sH3[2][kNW][64];   // H^{n+5/2} x, z of plane m-2
  __shared__ float sEzN[kNW];          // E_z at i = N of each row, current plane
  const int nb = a.nj * a.nk;
  const int lb = xcd_logical_block(nb);
  auto finish = [&]() {                // as in the two-step kernel, three steps
    if (threadIdx.x == 0) {
      if (atomicAdd(a.done, 1u) == gridDim.x - 1) {
        atomicExch(a.done, 0u);
        *a.step_w += 3;
      }
    }
  };
  if (lb >= nb) {
    finish();
    return;
  }
  const int tj = lb % a.nj, tkk = lb / a.nj;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int N = a.N, M = N + 1;
  const int i0 = NPL * lane;
  const int j = tj * kTJ - 3 + w;
  const int kb = tkk * a.tk, ke = min(kb + a.tk, M);   // output planes [kb, ke)
  const bool jv = j >= 0 && j <= N;
  const bool vld = jv && (FR || i0 <= N);
  const bool jup = vld && j + 1 <= N;
  const bool out = vld && w >= 3 && w < 3 + kTJ;
  const bool jj = j >= 1 && j <= N - 1, jlt = j < N;
  const bool last = lane == 63;
  const bool xn = FR && last && jv;
  // the rows (waves) that run phases B, C, D and E; F runs on the output rows
  const bool wB = w >= 1, wC = w >= 1 && w < kTJ + 4, wD = w >= 2 && w < kTJ + 4, wE = w >= 2 && w < kTJ + 3;
  auto iN = [&](int e) { return FR || i0 + e <= N; };
  auto ilt = [&](int e) { return FR || i0 + e < N; };
  auto ii = [&](int e) { return FR ? (e > 0 || lane > 0) : (i0 + e >= 1) & (i0 + e <= N - 1); };
  const bool srow = j == a.sj && a.si >= i0 && a.si < i0 + NPL;
  const int wm = w > 0 ? w - 1 : 0, wp = w < kNW - 1 ? w + 1 : kNW - 1;
  const size_t sk = (size_t)M * a.P;
  const unsigned pbytes = (unsigned)(M * a.P * 4);
  const unsigned ob = vld ? (unsigned)((j * a.P + i0) * 4) : kOff;
  const unsigned obj = jup ? (unsigned)(((j + 1) * a.P + i0) * 4) : kOff;
  const unsigned obN = xn ? (unsigned)((j * a.P + N) * 4) : kOff;
  // plane k of the input or output set: one resource for its six fields
  const unsigned span = (unsigned)(5 * a.fs) + pbytes;
  const int fs = (int)a.fs;
  auto pin = [&](int k) { return plane_rsrc(a.Ex + (size_t)k * sk, k >= 0 && k <= N ? span : 0u); };
  auto pout = [&](int k) { return plane_rsrc(a.oEx + (size_t)k * sk, k >= 0 && k <= N ? span : 0u); };
  enum { kEx, kEy, kEz, kHx, kHy, kHz };
  const float dt = a.dt;
  const long long n = *a.step;
  const bool add0 = n >= 0 && n < a.glen, add1 = n + 1 >= 0 && n + 1 < a.glen, add2 = n + 2 >= 0 && n + 2 < a.glen;
  const float g0 = add0 ? a.g[n] : 0.f, g1 = add1 ? a.g[n + 1] : 0.f, g2 = add2 ? a.g[n + 2] : 0.f;
  const Q z4{};
  auto ld = [&](int f, int k) -> Q { return qld_f<NPL>(pin(k), ob, f * fs); };
  auto ldj = [&](int f, int k) -> Q { return qld_f<NPL>(pin(k), obj, f * fs); };   // row j+1
  auto ldN = [&](int f, int k) -> float { return f1ld_f(pin(k), obN, f * fs); };
  // the source node's E_z after an E update: add the amplitude; the block
  // that outputs plane k records the probe
  auto source = [&](Q &ez_new, int k, bool add, float g, long long t) {
    if (k == a.sk) {
#pragma unroll
      for (int e = 0; e < NPL; ++e)
        if (srow && i0 + e == a.si) {
          if (add) ez_new.v[e] = ez_new.v[e] + g;
          if (out && k >= kb && k < ke && t >= 0 && t < a.pcap) a.probe[t] = ez_new.v[e];
        }
    }
  };

  const int m0 = max(kb - 3, 0);
  Q ex = ld(kEx, m0), ey = ld(kEy, m0), ez = ld(kEz, m0);   // E^n of plane m
  float eyN = ldN(kEy, m0), ezN = ldN(kEz, m0);               // E at i = N: plane m,
  float eyN_p = 0.f, ezN_p = 0.f, eyN_pp = 0.f, ezN_pp = 0.f;   // m-1, m-2
  Q h1x_p = z4, h1y_p = z4, h1z_p = z4;       // H^{n+1/2} of plane m-1
  Q e1y_p = z4;                               // E^{n+1}_y of plane m-1 (x, z: in sE1)
  Q h2x_p = z4, h2y_p = z4, h2z_p = z4;       // H^{n+3/2} of plane m-2
  Q e2y_p = z4;                               // E^{n+2}_y of plane m-2 (x, z: in sE2)
  Q h3x_p = z4, h3y_p = z4;                   // H^{n+5/2} of plane m-3
  // E^n of plane m+1, row j+1 of E^n and H of plane m, loaded one iteration ahead
  Q pexk = ld(kEx, m0 + 1), peyk = ld(kEy, m0 + 1), pezk = ld(kEz, m0 + 1);
  Q pex_j = ldj(kEx, m0), pez_j = ldj(kEz, m0);
  Q phx = ld(kHx, m0), phy = ld(kHy, m0), phz = ld(kHz, m0);
  float peyNk = ldN(kEy, m0 + 1), pezNk = ldN(kEz, m0 + 1), phxN = ldN(kHx, m0);
  for (int m = m0; m <= ke + 1; ++m) {
    const bool pm = m <= N;
    const Q exk = pexk, eyk = peyk, ezk = pezk, ex_j = pex_j, ez_j = pez_j, hx = phx, hy = phy, hz = phz;
    const float eyNk = peyNk, ezNk = pezNk, hxN = phxN;
    // ---- A: H^{n+1/2} of plane m
    const bool mlt = m < N;
    const Q ey_e = qeast(ey, last, eyN), ez_e = qeast(ez, last, ezN);
    Q h1x, h1y, h1z;
#pragma unroll
    for (int e = 0; e < NPL; ++e) {
      const float ux = hx.v[e] - dt * ((ez_j.v[e] - ez.v[e]) - (eyk.v[e] - ey.v[e]));
      const float uy = hy.v[e] - dt * ((exk.v[e] - ex.v[e]) - (ez_e.v[e] - ez.v[e]));
      const float uz = hz.v[e] - dt * ((ey_e.v[e] - ey.v[e]) - (ex_j.v[e] - ex.v[e]));
      h1x.v[e] = (iN(e) & jlt & mlt) ? ux : hx.v[e];
      h1y.v[e] = (ilt(e) & mlt) ? uy : hy.v[e];
      h1z.v[e] = (ilt(e) & jlt) ? uz : hz.v[e];
    }
    sH1[0][w][lane] = ldsof(h1x);
    sH1[1][w][lane] = ldsof(h1z);
    if (last) sEzN[w] = ezN;
    __syncthreads();                                         // ---- barrier 1
    {   // Hx at i = N of plane m: three updates with the column's unchanging E
      const float d = (sEzN[wp] - ezN) - (eyNk - eyN);
      const float h1 = hxN - dt * d;
      const float h2 = h1 - dt * d;
      const float h = (jlt & mlt) ? h2 - dt * d : hxN;
      const unsigned o = out && m >= kb && m < ke ? obN : kOff;
      f1st_f(pout(m), o, kHx * fs, h);
    }
    // ---- B: E^{n+1} of plane m
    Q e1x = z4, e1y = z4, e1z = z4;
    if (wB && pm) {
      const Q h1x_jm = qof(sH1[0][wm][lane]), h1z_jm = qof(sH1[1][wm][lane]);
      const Q h1z_w = qwest(h1z), h1y_w = qwest(h1y);
      const bool kk = m >= 1 && m <= N - 1;
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        const float ux = ex.v[e] + dt * ((h1z.v[e] - h1z_jm.v[e]) - (h1y.v[e] - h1y_p.v[e]));
        const float uy = ey.v[e] + dt * ((h1x.v[e] - h1x_p.v[e]) - (h1z.v[e] - h1z_w.v[e]));
        const float uz = ez.v[e] + dt * ((h1y.v[e] - h1y_w.v[e]) - (h1x.v[e] - h1x_jm.v[e]));
        e1x.v[e] = (ilt(e) & jj & kk) ? ux : ex.v[e];
        e1y.v[e] = (jlt & ii(e) & kk) ? uy : ey.v[e];
        e1z.v[e] = (mlt & ii(e) & jj) ? uz : ez.v[e];
      }
      source(e1z, m, add0, g0, n);
    }
    // ---- C: H^{n+3/2} of plane q = m-1 (E^{n+1} of row j+1, plane q, in sE1)
    const int q = m - 1;
    const bool doC = wC && q >= 0 && q >= kb - 2 && q <= ke;
    Q h2x = z4, h2y = z4, h2z = z4;
    // E^{n+1} x, z of plane q: this row's from sE1 (held there until barrier 3)
    const Q e1x_p = qof(sE1[0][w][lane]), e1z_p = qof(sE1[1][w][lane]);
    if (doC) {
      const Q e1x_jq = qof(sE1[0][wp][lane]), e1z_jq = qof(sE1[1][wp][lane]);
      const Q e1z_e = qeast(e1z_p, last, ezN_p), e1y_e = qeast(e1y_p, last, eyN_p);
      const bool qlt = q < N;
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        const float ux = h1x_p.v[e] - dt * ((e1z_jq.v[e] - e1z_p.v[e]) - (e1y.v[e] - e1y_p.v[e]));
        const float uy = h1y_p.v[e] - dt * ((e1x.v[e] - e1x_p.v[e]) - (e1z_e.v[e] - e1z_p.v[e]));
        const float uz = h1z_p.v[e] - dt * ((e1y_e.v[e] - e1y_p.v[e]) - (e1x_jq.v[e] - e1x_p.v[e]));
        h2x.v[e] = (iN(e) & jlt & qlt) ? ux : h1x_p.v[e];
        h2y.v[e] = (ilt(e) & qlt) ? uy : h1y_p.v[e];
        h2z.v[e] = (ilt(e) & jlt) ? uz : h1z_p.v[e];
      }
    }
    if (wC) {
      sH2[0][w][lane] = ldsof(h2x);
      sH2[1][w][lane] = ldsof(h2z);
    }
    __syncthreads();                                         // ---- barrier 2
    // the next plane's operands, issued here (half an iteration ahead) to
    // keep their registers free during A-C
    pexk = ld(kEx, m + 2); peyk = ld(kEy, m + 2); pezk = ld(kEz, m + 2);
    pex_j = ldj(kEx, m + 1); pez_j = ldj(kEz, m + 1);
    phx = ld(kHx, m + 1); phy = ld(kHy, m + 1); phz = ld(kHz, m + 1);
    peyNk = ldN(kEy, m + 2); pezNk = ldN(kEz, m + 2); phxN = ldN(kHx, m + 1);
    // ---- D: E^{n+2} of plane q
    Q e2x = z4, e2y = z4, e2z = z4;
    if (wD && doC && q <= N) {
      const Q h2x_jm = qof(sH2[0][wm][lane]), h2z_jm = qof(sH2[1][wm][lane]);
      const Q h2z_w = qwest(h2z), h2y_w = qwest(h2y);
      const bool kq = q >= 1 && q <= N - 1;
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        const float ux = e1x_p.v[e] + dt * ((h2z.v[e] - h2z_jm.v[e]) - (h2y.v[e] - h2y_p.v[e]));
        const float uy = e1y_p.v[e] + dt * ((h2x.v[e] - h2x_p.v[e]) - (h2z.v[e] - h2z_w.v[e]));
        const float uz = e1z_p.v[e] + dt * ((h2y.v[e] - h2y_w.v[e]) - (h2x.v[e] - h2x_jm.v[e]));
        e2x.v[e] = (ilt(e) & jj & kq) ? ux : e1x_p.v[e];
        e2y.v[e] = (jlt & ii(e) & kq) ? uy : e1y_p.v[e];
        e2z.v[e] = ((q < N) & ii(e) & jj) ? uz : e1z_p.v[e];
      }
      source(e2z, q, add1, g1, n + 1);
    }
    // ---- E: H^{n+5/2} of plane r = m-2 (E^{n+2} of row j+1, plane r, in sE2)
    const int r = m - 2;
    const bool doE = wE && r >= 0 && r >= kb - 1 && r <= ke - 1;
    Q h3x = z4, h3y = z4, h3z = z4;
    // E^{n+2} x, z of plane r: this row's from sE2 (held there until the end)
    const Q e2x_p = qof(sE2[0][w][lane]), e2z_p = qof(sE2[1][w][lane]);
    if (doE) {
      const Q e2x_jr = qof(sE2[0][wp][lane]), e2z_jr = qof(sE2[1][wp][lane]);
      const Q e2z_e = qeast(e2z_p, last, ezN_pp), e2y_e = qeast(e2y_p, last, eyN_pp);
      const bool rlt = r < N;
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        const float ux = h2x_p.v[e] - dt * ((e2z_jr.v[e] - e2z_p.v[e]) - (e2y.v[e] - e2y_p.v[e]));
        const float uy = h2y_p.v[e] - dt * ((e2x.v[e] - e2x_p.v[e]) - (e2z_e.v[e] - e2z_p.v[e]));
        const float uz = h2z_p.v[e] - dt * ((e2y_e.v[e] - e2y_p.v[e]) - (e2x_jr.v[e] - e2x_p.v[e]));
        h3x.v[e] = (iN(e) & jlt & rlt) ? ux : h2x_p.v[e];
        h3y.v[e] = (ilt(e) & rlt) ? uy : h2y_p.v[e];
        h3z.v[e] = (ilt(e) & jlt) ? uz : h2z_p.v[e];
      }
    }
    if (wE) {
      sH3[0][w][lane] = ldsof(h3x);
      sH3[1][w][lane] = ldsof(h3z);
    }
    __syncthreads();                                         // ---- barrier 3
    if (wB) {
      sE1[0][w][lane] = ldsof(e1x);                          // plane m: C, D of m+1
      sE1[1][w][lane] = ldsof(e1z);
    }
    // ---- F: E^{n+3} of plane r, and the outputs of plane r
    if (w >= 3 && w < kTJ + 3 && r >= kb && r <= ke - 1) {
      const Q h3x_jm = qof(sH3[0][wm][lane]), h3z_jm = qof(sH3[1][wm][lane]);
      const Q h3z_w = qwest(h3z), h3y_w = qwest(h3y);
      const bool kr = r >= 1 && r <= N - 1;
      Q e3x, e3y, e3z;
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        const float ux = e2x_p.v[e] + dt * ((h3z.v[e] - h3z_jm.v[e]) - (h3y.v[e] - h3y_p.v[e]));
        const float uy = e2y_p.v[e] + dt * ((h3x.v[e] - h3x_p.v[e]) - (h3z.v[e] - h3z_w.v[e]));
        const float uz = e2z_p.v[e] + dt * ((h3y.v[e] - h3y_w.v[e]) - (h3x.v[e] - h3x_jm.v[e]));
        e3x.v[e] = (ilt(e) & jj & kr) ? ux : e2x_p.v[e];
        e3y.v[e] = (jlt & ii(e) & kr) ? uy : e2y_p.v[e];
        e3z.v[e] = ((r < N) & ii(e) & jj) ? uz : e2z_p.v[e];
      }
      source(e3z, r, add2, g2, n + 2);
      const unsigned o = out ? ob : kOff;
      const __amdgpu_buffer_rsrc_t po = pout(r);
      qst_f<NT>(po, o, kEx * fs, e3x);
      qst_f<NT>(po, o, kEy * fs, e3y);
      qst_f<NT>(po, o, kEz * fs, e3z);
      qst_f<NT>(po, o, kHx * fs, h3x);
      qst_f<NT>(po, o, kHy * fs, h3y);
      qst_f<NT>(po, o, kHz * fs, h3z);
    }
    if (wD) {
      sE2[0][w][lane] = ldsof(e2x);                          // plane q: E, F of m+1
      sE2[1][w][lane] = ldsof(e2z);
    }
    // ---- rotate: plane m becomes the previous plane
    h3x_p = h3x; h3y_p = h3y;
    h2x_p = h2x; h2y_p = h2y; h2z_p = h2z;
    e2y_p = e2y;
    h1x_p = h1x; h1y_p = h1y; h1z_p = h1z;
    e1y_p = e1y;
    ex = exk; ey = eyk; ez = ezk;
    eyN_pp = eyN_p; ezN_pp = ezN_p;
    eyN_p = eyN; ezN_p = ezN;
    eyN = eyNk; ezN = ezNk;
  }
  finish();
}

bool make_fdtd_tb3_rows(Launch &L, const FdtdTbArgs &a0, bool nt) {
  FdtdTbArgs a = a0;
  const int M = a.N + 1;
  if (a.N > 4 * 64 || a.P % 4 != 0) return false;
  // the kernel addresses the fields as base + f * fs
  const float *in[6] = {a.Ex, a.Ey, a.Ez, a.Hx, a.Hy, a.Hz}, *out[6] = {a.oEx, a.oEy, a.oEz, a.oHx, a.oHy, a.oHz};
  for (int f = 0; f < 6; ++f)
    if ((const char *)in[f] != (const char *)a.Ex + f * a.fs || (const char *)out[f] != (const char *)a.oEx + f * a.fs)
      return false;
  constexpr int nw = 12;
  a.ni = 1;
  a.nj = (M + nw - 6) / (nw - 5);
  a.nk = std::max(1, std::min(kCUs / a.nj, M / 8));
  a.tk = (M + a.nk - 1) / a.nk;
  a.nk = (M + a.tk - 1) / a.tk;
  const int nb = a.nj * a.nk;
  // two nodes per lane up to N = 128 (a row of 129 nodes fills the wave),
  // four above
  const void *f;
  if (a.N <= 2 * 64) {
    const bool fr = a.N == 2 * 64;
    f = fr ? (nt ? (const void *)fdtd_tb3_rows_kernel<true, true, 2> : (const void *)fdtd_tb3_rows_kernel<false, true, 2>)
           : (nt ? (const void *)fdtd_tb3_rows_kernel<true, false, 2> : (const void *)fdtd_tb3_rows_kernel<false, false, 2>);
  } else {
    const bool fr = a.N == 4 * 64;
    f = fr ? (nt ? (const void *)fdtd_tb3_rows_kernel<true, true, 4> : (const void *)fdtd_tb3_rows_kernel<false, true, 4>)
           : (nt ? (const void *)fdtd_tb3_rows_kernel<true, false, 4> : (const void *)fdtd_tb3_rows_kernel<false, false, 4>);
  }
  L.set(f, dim3((unsigned)xcd_padded_grid(nb)), dim3(64 * nw), 0, a);
  return true;
}

struct StepAddArgs {
  long long *step;
  int d;
};

__global__ void fdtd_step_add_kernel(const StepAddArgs a) {
  if (threadIdx.x == 0) *a.step += a.d;
}

void make_fdtd_step_add(Launch &L, long long *step, int d) {
  L.set((const void *)fdtd_step_add_kernel, dim3(1), dim3(64), 0, StepAddArgs{step, d});
}

__global__ void fdtd_src_kernel(const SrcArgs s) {
  if (threadIdx.x != 0) return;
  const long long n = *s.step;
  float v = s.Ez[s.src];
  if (n >= 0 && n < s.glen) {
    v = v + s.g[n];
    s.Ez[s.src] = v;
  }
  if (n >= 0 && n < s.pcap) s.probe[n] = v;
  *s.step = n + 1;
}

void make_fdtd_src(Launch &L, const SrcArgs &a) { L.set((const void *)fdtd_src_kernel, dim3(1), dim3(64), 0, a); }

}  // namespace kb
