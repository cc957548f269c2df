// Thermal stencil kernels (2D 5-point, 3D 7-point, many-grid 2D) for gfx950.
//
// The update is the explicit thermal step of the Hotspot model that the
// paper batches (Sec. III-C):
//   T' = T + c*(P + (Tn+Ts-2T)/Ry + (Te+Tw-2T)/Rx [+ (Tu+Td-2T)/Rz] + (Tamb-T)/Rz)
// with neighbour indices clamped to the grid.  Every kernel evaluates it
// through heat_update*/ below in one fixed order of fused multiply-adds with
// the coefficients c, c/Rx, c/Ry, c/Rz pre-rounded to float, so all kernel
// variants (direct, LDS tile, temporal blocking, many-grid) produce the same
// bits for the same step.  The library is built with -ffp-contract=off, so
// only the explicit fmaf calls fuse.
//
// These kernels are bandwidth- or latency-bound (about 12 bytes and 13 flops
// per cell-step), so they use plain vector ALU work, coalesced row access
// (one wave64 covers 64 consecutive floats of a row) and LDS tiles, not MFMA.
#include "heat_update.h"
#include "kb_internal.h"

namespace kb {

// ---------------------------------------------------------------------------
// 2D direct kernel: one thread per cell, 64x4 threads per block.
// ---------------------------------------------------------------------------
constexpr int kDX = 64, kDY = 4;

__global__ __launch_bounds__(256) void heat2d_direct_kernel(const Heat2DArgs a) {
  const int tiles_x = (a.nx + kDX - 1) / kDX;
  const int tiles_y = (a.ny + kDY - 1) / kDY;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int j = (lb % tiles_x) * kDX + threadIdx.x;
  const int i = (lb / tiles_x) * kDY + threadIdx.y;
  if (i >= a.ny || j >= a.nx) return;
  const size_t nx = (size_t)a.nx;
  const int in = i > 0 ? i - 1 : 0;
  const int is = i < a.ny - 1 ? i + 1 : a.ny - 1;
  const int jw = j > 0 ? j - 1 : 0;
  const int je = j < a.nx - 1 ? j + 1 : a.nx - 1;
  const float *row = a.T + (size_t)i * nx;
  const float t = row[j];
  const float v = heat_update(t, a.T[(size_t)in * nx + j], a.T[(size_t)is * nx + j], row[jw], row[je],
                              a.P[(size_t)i * nx + j], a.k);
  a.out[(size_t)i * nx + j] = v;
}

void make_heat2d_direct(Launch &L, const Heat2DArgs &a) {
  int nb = ((a.nx + kDX - 1) / kDX) * ((a.ny + kDY - 1) / kDY);
  L.set((const void *)heat2d_direct_kernel, dim3(xcd_padded_grid(nb)), dim3(kDX, kDY), 0, a);
}

// ---------------------------------------------------------------------------
// 2D LDS tile kernel with temporal blocking.  A block owns a BX x BY tile of
// outputs.  It loads the tile plus a halo of t cells (clipped to the grid)
// into LDS, applies t steps there (ping-pong between two LDS buffers, P kept
// in a third), and writes the tile.  At the grid's own edges the neighbour
// index is clamped exactly as in a single step; at the halo's inner edges
// the clamp is wrong, but that error moves inward one cell per step and
// never reaches the tile after t steps.  Each step applies heat_update to
// every cell, so the result equals t direct steps bit for bit.
// ---------------------------------------------------------------------------
constexpr int kMaxDepth = 16;

template <int BX, int BY>
__global__ __launch_bounds__(BX *BY) void heat2d_tile_kernel(const Heat2DArgs a) {
  extern __shared__ float sm[];
  if (a.flag && *a.flag == 0) return;           // predicated launch (whole grid)
  const int t = a.tdepth;
  const int tiles_x = (a.nx + BX - 1) / BX;
  const int tiles_y = (a.ny + BY - 1) / BY;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int x0 = (lb % tiles_x) * BX;
  const int y0 = (lb / tiles_x) * BY;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + BX + t, a.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + BY + t, a.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo;
  const int cap = (BX + 2 * t) * (BY + 2 * t);
  float *A = sm;
  float *B = sm + cap;
  float *Ps = sm + 2 * cap;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const size_t nx = (size_t)a.nx;

  for (int yy = ty; yy < H; yy += BY) {
    const size_t g = (size_t)(ry_lo + yy) * nx + rx_lo;
    for (int xx = tx; xx < W; xx += BX) {
      A[yy * W + xx] = a.T[g + xx];
      Ps[yy * W + xx] = a.P[g + xx];
    }
  }
  __syncthreads();
  for (int s = 0; s < t; ++s) {
    for (int yy = ty; yy < H; yy += BY) {
      const int yn = yy > 0 ? yy - 1 : 0;
      const int ys = yy < H - 1 ? yy + 1 : H - 1;
      for (int xx = tx; xx < W; xx += BX) {
        const int xw = xx > 0 ? xx - 1 : 0;
        const int xe = xx < W - 1 ? xx + 1 : W - 1;
        B[yy * W + xx] = heat_update(A[yy * W + xx], A[yn * W + xx], A[ys * W + xx], A[yy * W + xw],
                                     A[yy * W + xe], Ps[yy * W + xx], a.k);
      }
    }
    __syncthreads();
    float *tmp = A; A = B; B = tmp;
  }
  const int gy = y0 + ty;
  for (int yy = gy; yy < min(y0 + BY, a.ny); yy += BY) {
    for (int xx = x0 + tx; xx < min(x0 + BX, a.nx); xx += BX) {
      a.out[(size_t)yy * nx + xx] = A[(yy - ry_lo) * W + (xx - rx_lo)];
    }
  }
}

template <int BX, int BY>
static void set_tile(Launch &L, const Heat2DArgs &a) {
  int nb = ((a.nx + BX - 1) / BX) * ((a.ny + BY - 1) / BY);
  unsigned shm = 3u * (BX + 2 * a.tdepth) * (BY + 2 * a.tdepth) * sizeof(float);
  L.set((const void *)heat2d_tile_kernel<BX, BY>, dim3(xcd_padded_grid(nb)), dim3(BX, BY), shm, a);
}

int heat2d_tile_max_depth() { return kMaxDepth; }

// ---------------------------------------------------------------------------
// Register-strip temporal blocking (variants 15, 16, 17): 16x16 output
// tiles, t <= 8 steps per launch over the tile grown by t cells on each
// side (at most 32x32, clamped to the grid).  Thread (g, cx) = (tid / 32,
// tid % 32) keeps RPT = 4, 2 or 1 rows RPT*g .. RPT*g+RPT-1 of region column
// cx in registers (256, 512 or 1024 threads): east / west neighbours come
// from the adjacent lanes by whole-wave DPP shifts (the value that crosses
// between the two 32-lane halves of a wave lands on a column the clamps
// replace), north / south from its own registers except at the strip ends,
// which are exchanged through LDS (double buffered: one barrier per step).
// Cells near a cut halo see a clamped neighbour; the error moves inward one
// cell per step and never reaches the tile.  Same update, same bits as
// every other variant.
// ---------------------------------------------------------------------------
constexpr int kStMaxDepth = 8;                // 32-column regions

// CWID = region columns (32 or 64); tiles of CWID/2 x CWID/2 cells, so
// t <= CWID/4; CWID/RPT row groups of CWID lanes.  With CWID = 64 a wave is
// one row group, and the 32 x 32 tiles allow 16 steps per launch.
template <int RPT, int CWID>
__global__ __launch_bounds__(CWID * (CWID / RPT)) void heat2d_strip_tb_kernel(const Heat2DArgs a) {
  constexpr int NG = CWID / RPT;               // row groups
  constexpr int TX = CWID / 2;                 // tile side
  __shared__ float ends[2][2][NG][CWID];       // [buffer][top, bottom][group][column]
  if (a.flag && *a.flag == 0) return;          // predicated launch (whole grid)
  const int t = a.tdepth;
  const int tiles_x = (a.nx + TX - 1) / TX, tiles_y = (a.ny + TX - 1) / TX;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int x0 = (lb % tiles_x) * TX, y0 = (lb / tiles_x) * TX;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + TX + t, a.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + TX + t, a.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo;
  const int cx = threadIdx.x % CWID, g = threadIdx.x / CWID, r0 = RPT * g;
  const int col = cx < W ? cx : W - 1;
  const size_t nx = (size_t)a.nx;
  float v[RPT], pw[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = r0 + i < H ? r0 + i : H - 1;
    const size_t gi = (size_t)(ry_lo + r) * nx + rx_lo + col;
    v[i] = a.T[gi];
    pw[i] = a.P[gi];
  }
  ends[0][0][g][cx] = v[0];
  ends[0][1][g][cx] = v[RPT - 1];
  __syncthreads();
  // one step from x to o, strip ends read from LDS buffer b, written to b^1
  auto step = [&](const float (&x)[RPT], float (&o)[RPT], int b) {
    // north of row r0 and south of row r0+RPT-1 (clamped at the region edge)
    const float top = g > 0 ? ends[b][1][g - 1][cx] : x[0];
    const float bot = g < NG - 1 ? ends[b][0][g + 1][cx] : x[RPT - 1];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + i;
      float wv = lane_west_open(x[i]), ev = lane_east_open(x[i]);
      if (cx == 0) wv = x[i];
      if (cx >= W - 1) ev = x[i];
      const float n = r == 0 ? x[i] : (i == 0 ? top : x[i - 1]);
      const float so = r >= H - 1 ? x[i] : (i == RPT - 1 ? bot : x[i + 1]);
      o[i] = heat_update(x[i], n, so, wv, ev, pw[i], a.k);
    }
    ends[b ^ 1][0][g][cx] = o[0];
    ends[b ^ 1][1][g][cx] = o[RPT - 1];
    __syncthreads();
  };
  // two steps at a time between two register sets (no register copies)
  float u[RPT];
  int s = 0;
  for (; s + 2 <= t; s += 2) {
    step(v, u, 0);
    step(u, v, 1);
  }
  if (s < t) {
    step(v, u, 0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = u[i];
  }
  if (cx < W) {
    const int gx = rx_lo + cx;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int gy = ry_lo + r0 + i;
      if (r0 + i < H && gy >= y0 && gy < y0 + TX && gx >= x0 && gx < x0 + TX) a.out[(size_t)gy * nx + gx] = v[i];
    }
  }
}

// variant 15: 4 rows per thread, 16: 2, 17: 1 (32-column regions, t <= 8);
// 22: 4 rows per thread, 23: 8 (64-column regions, t <= 16)
bool make_heat2d_strip(Launch &L, const Heat2DArgs &a, int variant) {
  const int cw = variant >= 22 ? 64 : 32;
  if (a.tdepth < 1 || a.tdepth > cw / 4) return false;
  const int tx = cw / 2;
  const int nb = ((a.nx + tx - 1) / tx) * ((a.ny + tx - 1) / tx);
  const dim3 grid(xcd_padded_grid(nb));
  if (variant == 15) L.set((const void *)heat2d_strip_tb_kernel<4, 32>, grid, dim3(256), 0, a);
  else if (variant == 16) L.set((const void *)heat2d_strip_tb_kernel<2, 32>, grid, dim3(512), 0, a);
  else if (variant == 17) L.set((const void *)heat2d_strip_tb_kernel<1, 32>, grid, dim3(1024), 0, a);
  else if (variant == 22) L.set((const void *)heat2d_strip_tb_kernel<4, 64>, grid, dim3(1024), 0, a);
  else if (variant == 23) L.set((const void *)heat2d_strip_tb_kernel<8, 64>, grid, dim3(512), 0, a);
  else return false;
  return true;
}
int heat2d_strip_max_depth() { return kStMaxDepth; }

// variant: 2 = 64x4, 3 = 64x8, 4 = 64x16, 5 = 32x8, 6 = 16x16, 7 = 32x4
bool make_heat2d_tile(Launch &L, const Heat2DArgs &a, int variant) {
  if (a.tdepth < 1 || a.tdepth > kMaxDepth) return false;
  switch (variant) {
    case 2: set_tile<64, 4>(L, a); return true;
    case 3: set_tile<64, 8>(L, a); return true;
    case 4: set_tile<64, 16>(L, a); return true;
    case 5: set_tile<32, 8>(L, a); return true;
    case 6: set_tile<16, 16>(L, a); return true;
    case 7: set_tile<32, 4>(L, a); return true;
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// Vector row kernels (rows of nx % 4 == 0 floats, so every row starts on a
// 16-byte boundary).  A wave64 covers 256 consecutive columns, four per lane
// as one float4; east/west neighbours come from the adjacent lanes through
// wave shuffles, and lanes 0 and 63 load the single cell beyond their wave
// (clamped at the grid edge).  Each wave walks R rows downwards keeping the
// rows above, at and below the current one in registers, so a row of T is
// read from memory once per strip plus one halo row at each end.
// ---------------------------------------------------------------------------
// Load of a float4 row segment read once per step (the power map P): with
// NT, a non-temporal (streaming) load, as the streaming-store variants use
// for data that no other wave of the step reads again.
template <bool NT>
__device__ __forceinline__ float4 load_once4(const float *base, size_t row, size_t nx, int x, bool xin) {
  if (!xin) return make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (NT) {
    typedef float f4l __attribute__((ext_vector_type(4)));
    const f4l v = __builtin_nontemporal_load(reinterpret_cast<const f4l *>(base + row * nx + x));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *reinterpret_cast<const float4 *>(base + row * nx + x);
  }
}

__device__ __forceinline__ float4 load_row4(const float *base, size_t row, size_t nx, int x, bool xin) {
  return xin ? *reinterpret_cast<const float4 *>(base + row * nx + x) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// West and east neighbours of a lane's four cells in one row.
__device__ __forceinline__ void row_neighbours(const float *row, const float4 &c, int x, int nx, int lane,
                                               float &wv, float &ev) {
  wv = lane_west_open(c.w);
  ev = lane_east_open(c.x);
  if (lane == 0) wv = x > 0 ? row[x - 1] : c.x;
  if (x + 4 >= nx) ev = c.w;
  else if (lane == 63) ev = row[x + 4];
}

// The same neighbours with the two loads apart: `load_row_edges` reads the
// value west of lane 0 and east of lane 63 (issued with the loads of the
// next layer, so that waiting for them does not also wait for loads issued
// after them), `edge_neighbours` combines them with the lane shifts.
struct RowEdges {
  float w, e;
};
__device__ __forceinline__ RowEdges load_row_edges(const float *row, int x, int nx, int lane) {
  RowEdges g{0.f, 0.f};
  if (lane == 0 && x > 0) g.w = row[x - 1];
  if (lane == 63 && x + 4 < nx) g.e = row[x + 4];
  return g;
}
__device__ __forceinline__ void edge_neighbours(const RowEdges &g, const float4 &c, int x, int nx, int lane,
                                                float &wv, float &ev) {
  wv = lane_west_open(c.w);
  ev = lane_east_open(c.x);
  if (lane == 0) wv = x > 0 ? g.w : c.x;
  if (x + 4 >= nx) ev = c.w;
  else if (lane == 63) ev = g.e;
}

typedef float f4v __attribute__((ext_vector_type(4)));

// Store a float4 row segment; NT = non-temporal (streaming) store that does
// not keep the line in cache.
template <bool NT>
__device__ __forceinline__ void store_row4(float *__restrict__ dst, const float4 &o) {
  if constexpr (NT) {
    f4v v = {o.x, o.y, o.z, o.w};
    __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(dst));
  } else {
    *reinterpret_cast<float4 *>(dst) = o;
  }
}

template <int R, bool NT>
__global__ __launch_bounds__(256) void heat2d_vec_kernel(const Heat2DArgs a) {
  const int tiles_x = (a.nx + 255) / 256;
  const int tiles_y = (a.ny + 4 * R - 1) / (4 * R);
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int lane = threadIdx.x;
  const int y0 = (lb / tiles_x) * (4 * R) + threadIdx.y * R;
  if (y0 >= a.ny) return;                       // whole wave
  const int x = (lb % tiles_x) * 256 + lane * 4;
  const bool xin = x < a.nx;
  const size_t nx = (size_t)a.nx;
  const float *__restrict__ T = a.T;            // T, P and out never alias
  const float *__restrict__ P = a.P;
  float *__restrict__ out = a.out;
  float4 up = load_row4(T, y0 > 0 ? y0 - 1 : 0, nx, x, xin);
  float4 cur = load_row4(T, y0, nx, x, xin);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = y0 + r;
    if (y >= a.ny) break;
    const float4 dn = load_row4(T, y + 1 < a.ny ? y + 1 : a.ny - 1, nx, x, xin);
    const float4 p = load_once4<NT>(P, y, nx, x, xin);
    float wv, ev;
    row_neighbours(T + (size_t)y * nx, cur, x, a.nx, lane, wv, ev);
    float4 o;
    o.x = heat_update(cur.x, up.x, dn.x, wv, cur.y, p.x, a.k);
    o.y = heat_update(cur.y, up.y, dn.y, cur.x, cur.z, p.y, a.k);
    o.z = heat_update(cur.z, up.z, dn.z, cur.y, cur.w, p.z, a.k);
    o.w = heat_update(cur.w, up.w, dn.w, cur.z, ev, p.w, a.k);
    if (xin) store_row4<NT>(out + (size_t)y * nx + x, o);
    up = cur;
    cur = dn;
  }
}

template <int R, bool NT>
static void set_vec(Launch &L, const Heat2DArgs &a) {
  int nb = ((a.nx + 255) / 256) * ((a.ny + 4 * R - 1) / (4 * R));
  L.set((const void *)heat2d_vec_kernel<R, NT>, dim3(xcd_padded_grid(nb)), dim3(64, 4), 0, a);
}

// variant: 8 = 1 row per wave, 9 = 2, 10 = 4, 11 = 8, 12 = 16;
//          13 = 1 row per wave with non-temporal stores, 14 = 2 rows, ditto
bool make_heat2d_vec(Launch &L, const Heat2DArgs &a, int variant) {
  if (a.nx % 4 != 0) return false;
  switch (variant) {
    case 8: set_vec<1, false>(L, a); return true;
    case 9: set_vec<2, false>(L, a); return true;
    case 10: set_vec<4, false>(L, a); return true;
    case 11: set_vec<8, false>(L, a); return true;
    case 12: set_vec<16, false>(L, a); return true;
    case 13: set_vec<1, true>(L, a); return true;
    case 14: set_vec<2, true>(L, a); return true;
    default: return false;
  }
}

// 3D vector kernel: a wave covers 256 columns of one row and marches up the
// layers with the layers below, at and above in registers; the rows y-1 and
// y+1 of the current layer are read (they are the rows of the neighbouring
// waves, so they come from cache).  PF: the loads of layer z+1 are issued
// before layer z is computed and stored (software pipelining), so every
// wave keeps the next layer's three rows in flight.  NT: streaming stores.
template <bool PF, bool NT>
__global__ __launch_bounds__(256) void heat3d_vec_kernel(const Heat3DArgs a) {
  const int tiles_x = (a.nx + 255) / 256;
  const int tiles_y = (a.ny + 3) / 4;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int lane = threadIdx.x;
  const int y = (lb / tiles_x) * 4 + threadIdx.y;
  if (y >= a.ny) return;
  const int x = (lb % tiles_x) * 256 + lane * 4;
  const bool xin = x < a.nx;
  const size_t nx = (size_t)a.nx;
  const size_t ny = (size_t)a.ny;
  const size_t yn = y > 0 ? y - 1 : 0, ys = y + 1 < a.ny ? y + 1 : a.ny - 1;
  const float *__restrict__ T = a.T;            // T, P and out never alias
  const float *__restrict__ P = a.P;
  float *__restrict__ out = a.out;
  float4 td = load_row4(T, y, nx, x, xin);
  float4 tc = td;
  // rows of layer 0 (and layer 1 above it) for the first iteration
  float4 tu = a.nz > 1 ? load_row4(T, ny + y, nx, x, xin) : tc;
  float4 tn = load_row4(T, yn, nx, x, xin);
  float4 ts = load_row4(T, ys, nx, x, xin);
  for (int z = 0; z < a.nz; ++z) {
    const size_t zr = (size_t)z * ny;            // first row of layer z
    if constexpr (!PF) {
      if (z > 0) {
        tu = z + 1 < a.nz ? load_row4(T, zr + ny + y, nx, x, xin) : tc;
        tn = load_row4(T, zr + yn, nx, x, xin);
        ts = load_row4(T, zr + ys, nx, x, xin);
      }
    }
    float4 tu2 = tu, tn2 = tn, ts2 = ts;         // rows for layer z+1
    if constexpr (PF) {
      if (z + 1 < a.nz) {
        tu2 = z + 2 < a.nz ? load_row4(T, zr + 2 * ny + y, nx, x, xin) : tu;
        tn2 = load_row4(T, zr + ny + yn, nx, x, xin);
        ts2 = load_row4(T, zr + ny + ys, nx, x, xin);
      }
    }
    const bool hp = z == 0;
    const float4 p = hp ? load_once4<NT>(P, y, nx, x, xin) : make_float4(0.f, 0.f, 0.f, 0.f);
    float wv, ev;
    row_neighbours(T + (zr + y) * nx, tc, x, a.nx, lane, wv, ev);
    float4 o;
    o.x = heat3d_update(tc.x, tn.x, ts.x, wv, tc.y, tu.x, td.x, p.x, hp, a.k);
    o.y = heat3d_update(tc.y, tn.y, ts.y, tc.x, tc.z, tu.y, td.y, p.y, hp, a.k);
    o.z = heat3d_update(tc.z, tn.z, ts.z, tc.y, tc.w, tu.z, td.z, p.z, hp, a.k);
    o.w = heat3d_update(tc.w, tn.w, ts.w, tc.z, ev, tu.w, td.w, p.w, hp, a.k);
    if (xin) store_row4<NT>(out + (zr + y) * nx + x, o);
    td = tc;
    tc = tu;
    if constexpr (PF) {
      tu = tu2;
      tn = tn2;
      ts = ts2;
    }
  }
}

// ---------------------------------------------------------------------------
// Register-blocked 3D rows: wave w of a block covers rows y0 .. y0+R-1 of
// 256 consecutive columns (a float4 per lane) and marches up the layers.
// For each layer it loads the R rows of the next layer together with the
// row above and the row below them -- R + 2 row loads for R output rows,
// where the one-row kernel issues three -- and keeps the layers below, at
// and above the current one in registers.  NT: streaming stores.  PF: the
// rows of the layer after next, and the values beyond the wave's ends in
// the next layer's rows, are loaded one iteration ahead.
// ---------------------------------------------------------------------------
template <int R, bool NT, bool PF>
__global__ __launch_bounds__(256) void heat3d_rows_kernel(const Heat3DArgs a) {
  const int tiles_x = (a.nx + 255) / 256;
  const int tiles_y = (a.ny + 4 * R - 1) / (4 * R);
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int lane = threadIdx.x;
  const int y0 = (lb / tiles_x) * (4 * R) + threadIdx.y * R;
  if (y0 >= a.ny) return;                       // uniform per wave
  const int x = (lb % tiles_x) * 256 + lane * 4;
  const bool xin = x < a.nx;
  const size_t nx = (size_t)a.nx, ny = (size_t)a.ny;
  const float *__restrict__ T = a.T;
  const float *__restrict__ P = a.P;
  float *__restrict__ out = a.out;
  size_t rows[R + 2];                           // rows y0-1 .. y0+R, clamped
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const int yy = y0 - 1 + r;
    rows[r] = (size_t)(yy < 0 ? 0 : (yy >= a.ny ? a.ny - 1 : yy));
  }
  float4 c[R + 2], u[R + 2], d[R], u2[R + 2];
  RowEdges eg[R], egn[R];                       // PF: ends of layer z, z+1
#pragma unroll
  for (int r = 0; r < R + 2; ++r) c[r] = load_row4(T, rows[r], nx, x, xin);
#pragma unroll
  for (int r = 0; r < R; ++r) d[r] = c[r + 1];  // below layer 0: itself
  if constexpr (PF) {                           // layer 1 rows, one layer ahead
#pragma unroll
    for (int r = 0; r < R + 2; ++r) u2[r] = a.nz > 1 ? load_row4(T, ny + rows[r], nx, x, xin) : c[r];
#pragma unroll
    for (int r = 0; r < R; ++r) eg[r] = load_row_edges(T + rows[r + 1] * nx, x, a.nx, lane);
  }
  for (int z = 0; z < a.nz; ++z) {
    const size_t zr = (size_t)z * ny;
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < R + 2; ++r) u[r] = u2[r];
      if (z + 2 < a.nz) {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) u2[r] = load_row4(T, zr + 2 * ny + rows[r], nx, x, xin);
      } else {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) u2[r] = u[r];
      }
      if (z + 1 < a.nz) {
#pragma unroll
        for (int r = 0; r < R; ++r) egn[r] = load_row_edges(T + (zr + ny + rows[r + 1]) * nx, x, a.nx, lane);
      }
      if (z + 1 >= a.nz) {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) u[r] = c[r];        // above the top layer: itself
      }
    } else {
      if (z + 1 < a.nz) {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) u[r] = load_row4(T, zr + ny + rows[r], nx, x, xin);
      } else {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) u[r] = c[r];        // above the top layer: itself
      }
    }
    const bool hp = z == 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int yy = y0 + r;
      if (yy < a.ny) {
        const float4 tc = c[r + 1], tn = c[r], ts = c[r + 2], tu = u[r + 1], td = d[r];
        const float4 p = hp ? load_once4<NT>(P, (size_t)yy, nx, x, xin) : make_float4(0.f, 0.f, 0.f, 0.f);
        float wv, ev;
        if constexpr (PF) edge_neighbours(eg[r], tc, x, a.nx, lane, wv, ev);
        else row_neighbours(T + (zr + yy) * nx, tc, x, a.nx, lane, wv, ev);
        float4 o;
        o.x = heat3d_update(tc.x, tn.x, ts.x, wv, tc.y, tu.x, td.x, p.x, hp, a.k);
        o.y = heat3d_update(tc.y, tn.y, ts.y, tc.x, tc.z, tu.y, td.y, p.y, hp, a.k);
        o.z = heat3d_update(tc.z, tn.z, ts.z, tc.y, tc.w, tu.z, td.z, p.z, hp, a.k);
        o.w = heat3d_update(tc.w, tn.w, ts.w, tc.z, ev, tu.w, td.w, p.w, hp, a.k);
        if (xin) store_row4<NT>(out + (zr + yy) * nx + x, o);
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < R; ++r) eg[r] = egn[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) d[r] = c[r + 1];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) c[r] = u[r];
  }
}

// ---------------------------------------------------------------------------
// 3D kernel: one thread per (x, y) column, marching up the layers with the
// column's three consecutive layers in registers.  P is the plane of layer 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void heat3d_kernel(const Heat3DArgs a) {
  const int tiles_x = (a.nx + kDX - 1) / kDX;
  const int tiles_y = (a.ny + kDY - 1) / kDY;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int j = (lb % tiles_x) * kDX + threadIdx.x;
  const int i = (lb / tiles_x) * kDY + threadIdx.y;
  if (i >= a.ny || j >= a.nx) return;
  const size_t nx = (size_t)a.nx;
  const size_t plane = (size_t)a.ny * nx;
  const int in = i > 0 ? i - 1 : 0;
  const int is = i < a.ny - 1 ? i + 1 : a.ny - 1;
  const int jw = j > 0 ? j - 1 : 0;
  const int je = j < a.nx - 1 ? j + 1 : a.nx - 1;
  const size_t c = (size_t)i * nx + j;
  const size_t on = (size_t)in * nx + j, os = (size_t)is * nx + j;
  const size_t ow = (size_t)i * nx + jw, oe = (size_t)i * nx + je;
  float td = a.T[c];
  float tc = td;
  for (int z = 0; z < a.nz; ++z) {
    const size_t base = (size_t)z * plane;
    const float tu = (z + 1 < a.nz) ? a.T[base + plane + c] : tc;
    const float p = (z == 0) ? a.P[c] : 0.0f;
    const float v = heat3d_update(tc, a.T[base + on], a.T[base + os], a.T[base + ow], a.T[base + oe], tu, td, p,
                                  z == 0, a.k);
    a.out[base + c] = v;
    td = tc;
    tc = tu;
  }
}

// ---------------------------------------------------------------------------
// Temporal blocking for layered stacks (nz <= 8): one launch advances t
// (<= 6) steps.  A block owns a 32x32 tile of columns and loads the tile grown by
// t columns on each side (clamped to the field) with all nz layers.  Each
// of the 512 threads keeps up to kTbCols whole columns (every layer) in
// registers; per
// step it publishes them to an LDS plane stack, then updates them from the
// four in-plane neighbours in LDS and the layers above and below in its own
// registers.  Region cells next to a cut halo see a clamped neighbour that
// is not the true one; the error moves inward one column per step and never
// reaches the tile.  Same update, same bits as the one-step kernels.
// ---------------------------------------------------------------------------
constexpr int kTbX = 32, kTbY = 32, kTbMaxDepth = 6;   // 8 layers x 44^2 floats <= 64 KB of LDS
constexpr int kTbThreads = 512;
constexpr int kTbCols = ((kTbX + 2 * kTbMaxDepth) * (kTbY + 2 * kTbMaxDepth) + kTbThreads - 1) / kTbThreads;   // 4

// deepest temporal blocking of any 3D variant (variant 5: 6, variant 11: 8;
// a launch checks its own variant's limit)
int heat3d_tb_max_depth() { return 8; }

template <int NZ>
__global__ __launch_bounds__(kTbThreads) void heat3d_tb_kernel(const Heat3DArgs a) {
  extern __shared__ float lds[];
  const int t = a.tdepth;
  const int tiles_x = (a.nx + kTbX - 1) / kTbX, tiles_y = (a.ny + kTbY - 1) / kTbY;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int x0 = (lb % tiles_x) * kTbX, y0 = (lb / tiles_x) * kTbY;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + kTbX + t, a.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + kTbY + t, a.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo, R = W * H;
  const size_t plane = (size_t)a.ny * a.nx;
  float v[kTbCols][NZ], p[kTbCols];
  int rc[kTbCols];                      // (row << 8) | col in the region
#pragma unroll
  for (int q = 0; q < kTbCols; ++q) {
    const int c = threadIdx.x + kTbThreads * q;
    const int cc = c < R ? c : R - 1;
    const int ry = cc / W, rx = cc - (cc / W) * W;
    rc[q] = (ry << 8) | rx;
    const size_t g = (size_t)(ry_lo + ry) * a.nx + rx_lo + rx;
#pragma unroll
    for (int z = 0; z < NZ; ++z) v[q][z] = a.T[z * plane + g];
    p[q] = a.P[g];
  }
  for (int s = 0; s < t; ++s) {
#pragma unroll
    for (int q = 0; q < kTbCols; ++q) {
      const int c = threadIdx.x + kTbThreads * q;
      if (c < R)
#pragma unroll
        for (int z = 0; z < NZ; ++z) lds[z * R + c] = v[q][z];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTbCols; ++q) {
      const int c = threadIdx.x + kTbThreads * q;
      const int ry = rc[q] >> 8, rx = rc[q] & 255;
      const int cc = ry * W + rx;
      const int on = ry > 0 ? cc - W : cc, os = ry < H - 1 ? cc + W : cc;
      const int ow = rx > 0 ? cc - 1 : cc, oe = rx < W - 1 ? cc + 1 : cc;
      float nv[NZ];
#pragma unroll
      for (int z = 0; z < NZ; ++z) {
        const float tc = v[q][z];
        const float tu = z + 1 < NZ ? v[q][z + 1] : tc;
        const float td = z > 0 ? v[q][z - 1] : tc;
        nv[z] = heat3d_update(tc, lds[z * R + on], lds[z * R + os], lds[z * R + ow], lds[z * R + oe], tu, td,
                              z == 0 ? p[q] : 0.0f, z == 0, a.k);
      }
      if (c < R)
#pragma unroll
        for (int z = 0; z < NZ; ++z) v[q][z] = nv[z];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kTbCols; ++q) {
    const int c = threadIdx.x + kTbThreads * q;
    const int ry = rc[q] >> 8, rx = rc[q] & 255;
    const int gy = ry_lo + ry, gx = rx_lo + rx;
    if (c < R && gy >= y0 && gy < y0 + kTbY && gx >= x0 && gx < x0 + kTbX) {
      const size_t g = (size_t)gy * a.nx + gx;
#pragma unroll
      for (int z = 0; z < NZ; ++z) a.out[z * plane + g] = v[q][z];
    }
  }
}

static const void *heat3d_tb_fn(int nz) {
  switch (nz) {
    case 1: return (const void *)heat3d_tb_kernel<1>;
    case 2: return (const void *)heat3d_tb_kernel<2>;
    case 3: return (const void *)heat3d_tb_kernel<3>;
    case 4: return (const void *)heat3d_tb_kernel<4>;
    case 5: return (const void *)heat3d_tb_kernel<5>;
    case 6: return (const void *)heat3d_tb_kernel<6>;
    case 7: return (const void *)heat3d_tb_kernel<7>;
    case 8: return (const void *)heat3d_tb_kernel<8>;
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// 3D register-strip temporal blocking (variant 11, nz <= 8): t <= 8 steps
// per launch.  Output tiles of (64 - 2t) x (32 - 2t) columns, each block of
// 8 waves loads its tile grown by t on each side (at most 64 x 32 columns,
// clamped to the grid) with every layer: wave w holds region rows
// 4w .. 4w+3 of column `lane`, all nz layers, in registers.  Vertical
// neighbours are the thread's own registers, east / west come from the
// adjacent lanes, north / south from the wave's registers except at its
// strip ends, which are exchanged through LDS (double buffered: one
// barrier per step).  As in the 2D kernels, only the region sides on a
// grid edge need the clamp, and the step loop is specialised on them.
// ---------------------------------------------------------------------------
constexpr int kH3Waves = 8, kH3Rows = 4, kH3RegionY = kH3Waves * kH3Rows, kH3MaxDepth = 8;
constexpr int kH3TwoSetBlocks = 256;

// One step of a region column's rows (every layer) from `a` to `o`, strip
// ends read from LDS buffer b and written to b^1.  Writing into other
// registers than the step reads keeps the old rows alive as the next row's
// north neighbours without register copies.
template <int NZ, bool CW, bool CE, bool CS>
__device__ __forceinline__ void heat3d_strip_step(const float (&a)[NZ][kH3Rows], float (&o)[NZ][kH3Rows],
                                                  const float (&pw)[kH3Rows],
                                                  float (*ends)[2][kH3Waves][NZ][64], int b, int W, int last,
                                                  int cx, int w, const HeatCoef &k) {
  float top[NZ], bot[NZ];
#pragma unroll
  for (int z = 0; z < NZ; ++z) {
    top[z] = w > 0 ? ends[b][1][w - 1][z][cx] : a[z][0];          // old row above
    bot[z] = w < kH3Waves - 1 ? ends[b][0][w + 1][z][cx] : a[z][kH3Rows - 1];
  }
#pragma unroll
  for (int i = 0; i < kH3Rows; ++i) {
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
      const float c = a[z][i];
      const float n = i == 0 ? top[z] : a[z][i - 1];
      float so = i == kH3Rows - 1 ? bot[z] : a[z][i + 1];
      if (CS && i == last) so = c;
      float ev = lane_east_open(c), wv = lane_west_open(c);
      if (CE && cx >= W - 1) ev = c;
      if (CW && cx == 0) wv = c;
      const float up = z + 1 < NZ ? a[z + 1][i] : c;
      const float dn = z > 0 ? a[z - 1][i] : c;
      o[z][i] = heat3d_update(c, n, so, wv, ev, up, dn, z == 0 ? pw[i] : 0.0f, z == 0, k);
    }
  }
#pragma unroll
  for (int z = 0; z < NZ; ++z) {
    ends[b ^ 1][0][w][z][cx] = o[z][0];
    ends[b ^ 1][1][w][z][cx] = o[z][kH3Rows - 1];
  }
  __syncthreads();
}

// t steps.  TWO: two at a time between two register sets (no register
// copies, but about 40 more VGPRs at NZ = 8, which halves the blocks per
// CU); otherwise one set, each step through a copy of the rows.
template <int NZ, bool TWO, bool CW, bool CE, bool CS>
__device__ __forceinline__ void heat3d_strip_advance(float (&v)[NZ][kH3Rows], const float (&pw)[kH3Rows],
                                                     float (*ends)[2][kH3Waves][NZ][64], int t, int W, int H,
                                                     int cx, int w, const HeatCoef &k) {
  const int last = H - 1 - kH3Rows * w;        // this wave's index of the grid's bottom row (CS)
  float u[NZ][kH3Rows];
  int s = 0;
  if constexpr (TWO) {
    for (; s + 2 <= t; s += 2) {
      heat3d_strip_step<NZ, CW, CE, CS>(v, u, pw, ends, 0, W, last, cx, w, k);
      heat3d_strip_step<NZ, CW, CE, CS>(u, v, pw, ends, 1, W, last, cx, w, k);
    }
  }
  int b = 0;
  for (; s < t; ++s) {
    heat3d_strip_step<NZ, CW, CE, CS>(v, u, pw, ends, b, W, last, cx, w, k);
    b ^= 1;
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int i = 0; i < kH3Rows; ++i) v[z][i] = u[z][i];
  }
}

template <int NZ, bool TWO>
__global__ __launch_bounds__(64 * kH3Waves) void heat3d_strip_tb_kernel(const Heat3DArgs a) {
  __shared__ float ends[2][2][kH3Waves][NZ][64];   // [buffer][top, bottom][wave][layer][column]
  const int t = a.tdepth, tile_x = 64 - 2 * t, tile_y = kH3RegionY - 2 * t;
  const int tiles_x = (a.nx + tile_x - 1) / tile_x, tiles_y = (a.ny + tile_y - 1) / tile_y;
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const int x0 = (lb % tiles_x) * tile_x, y0 = (lb / tiles_x) * tile_y;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + tile_x + t, a.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + tile_y + t, a.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo;
  const int cx = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int r0 = kH3Rows * w;
  const int col = cx < W ? cx : W - 1;
  const size_t nx = (size_t)a.nx, plane = (size_t)a.ny * nx;
  const size_t base = (size_t)ry_lo * nx + rx_lo;
  float v[NZ][kH3Rows], pw[kH3Rows];
#pragma unroll
  for (int i = 0; i < kH3Rows; ++i) {
    const int r = r0 + i < H ? r0 + i : H - 1;
    const size_t g = base + (size_t)r * nx + col;
#pragma unroll
    for (int z = 0; z < NZ; ++z) v[z][i] = a.T[z * plane + g];
    pw[i] = a.P[g];
  }
#pragma unroll
  for (int z = 0; z < NZ; ++z) {
    ends[0][0][w][z][cx] = v[z][0];
    ends[0][1][w][z][cx] = v[z][kH3Rows - 1];
  }
  __syncthreads();
  switch ((rx_lo == 0) | (rx_hi == a.nx) << 1 | (ry_hi == a.ny) << 2) {
    case 0: heat3d_strip_advance<NZ, TWO, false, false, false>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 1: heat3d_strip_advance<NZ, TWO, true, false, false>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 2: heat3d_strip_advance<NZ, TWO, false, true, false>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 3: heat3d_strip_advance<NZ, TWO, true, true, false>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 4: heat3d_strip_advance<NZ, TWO, false, false, true>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 5: heat3d_strip_advance<NZ, TWO, true, false, true>(v, pw, ends, t, W, H, cx, w, a.k); break;
    case 6: heat3d_strip_advance<NZ, TWO, false, true, true>(v, pw, ends, t, W, H, cx, w, a.k); break;
    default: heat3d_strip_advance<NZ, TWO, true, true, true>(v, pw, ends, t, W, H, cx, w, a.k); break;
  }
  const int gx = rx_lo + cx;
  if (cx < W && gx >= x0 && gx < x0 + tile_x) {
#pragma unroll
    for (int i = 0; i < kH3Rows; ++i) {
      const int gy = ry_lo + r0 + i;
      if (r0 + i < H && gy >= y0 && gy < y0 + tile_y) {
        const size_t g = (size_t)gy * nx + gx;
#pragma unroll
        for (int z = 0; z < NZ; ++z) a.out[z * plane + g] = v[z][i];
      }
    }
  }
}

static const void *heat3d_strip_fn(int nz, bool two) {
  switch (nz) {
    case 1: return two ? (const void *)heat3d_strip_tb_kernel<1, true> : (const void *)heat3d_strip_tb_kernel<1, false>;
    case 2: return two ? (const void *)heat3d_strip_tb_kernel<2, true> : (const void *)heat3d_strip_tb_kernel<2, false>;
    case 3: return two ? (const void *)heat3d_strip_tb_kernel<3, true> : (const void *)heat3d_strip_tb_kernel<3, false>;
    case 4: return two ? (const void *)heat3d_strip_tb_kernel<4, true> : (const void *)heat3d_strip_tb_kernel<4, false>;
    case 5: return two ? (const void *)heat3d_strip_tb_kernel<5, true> : (const void *)heat3d_strip_tb_kernel<5, false>;
    case 6: return two ? (const void *)heat3d_strip_tb_kernel<6, true> : (const void *)heat3d_strip_tb_kernel<6, false>;
    case 7: return two ? (const void *)heat3d_strip_tb_kernel<7, true> : (const void *)heat3d_strip_tb_kernel<7, false>;
    case 8: return two ? (const void *)heat3d_strip_tb_kernel<8, true> : (const void *)heat3d_strip_tb_kernel<8, false>;
  }
  return nullptr;
}

// variant: 1 = scalar columns; vector rows (nx % 4 == 0): 2 = plain,
// 3 = next layer prefetched, 4 = prefetched with streaming stores;
// 5 = temporal blocking over a.tdepth steps (nz <= 8); register-blocked
// rows with streaming stores (nx % 4 == 0): 6 = 2 rows, 7 = 4, 8 = 8 per
// wave; 9 = 2 rows, 10 = 4 rows, with the layer after next loaded ahead;
// 11 = register-strip temporal blocking (nz <= 8, a.tdepth <= 8)
bool make_heat3d(Launch &L, const Heat3DArgs &a, int variant) {
  if (variant == 11) {
    if (a.tdepth < 1 || a.tdepth > kH3MaxDepth) return false;
    const int tx = 64 - 2 * a.tdepth, ty = kH3RegionY - 2 * a.tdepth;
    const int nb = ((a.nx + tx - 1) / tx) * ((a.ny + ty - 1) / ty);
    // grids of at most one block per compute unit (256 on MI355X) take the
    // two-register-set loop: fewer instructions per step, and the blocks
    // per CU it costs are not needed
    const void *f = heat3d_strip_fn(a.nz, nb <= kH3TwoSetBlocks);
    if (!f) return false;
    L.set(f, dim3(xcd_padded_grid(nb)), dim3(64 * kH3Waves), 0, a);
    return true;
  }
  if (variant == 5) {
    const void *f = heat3d_tb_fn(a.nz);
    if (!f || a.tdepth < 1 || a.tdepth > kTbMaxDepth) return false;
    const int nb = ((a.nx + kTbX - 1) / kTbX) * ((a.ny + kTbY - 1) / kTbY);
    const unsigned lds = (unsigned)(a.nz * (kTbX + 2 * a.tdepth) * (kTbY + 2 * a.tdepth) * sizeof(float));
    L.set(f, dim3(xcd_padded_grid(nb)), dim3(kTbThreads), lds, a);
    return true;
  }
  if (variant >= 6 && variant <= 10) {
    if (a.nx % 4 != 0) return false;
    const int R = variant == 6 || variant == 9 ? 2 : variant == 7 || variant == 10 ? 4 : 8;
    const int nb = ((a.nx + 255) / 256) * ((a.ny + 4 * R - 1) / (4 * R));
    const void *f = variant == 6  ? (const void *)heat3d_rows_kernel<2, true, false>
                  : variant == 7  ? (const void *)heat3d_rows_kernel<4, true, false>
                  : variant == 8  ? (const void *)heat3d_rows_kernel<8, true, false>
                  : variant == 9  ? (const void *)heat3d_rows_kernel<2, true, true>
                                  : (const void *)heat3d_rows_kernel<4, true, true>;
    L.set(f, dim3(xcd_padded_grid(nb)), dim3(64, 4), 0, a);
    return true;
  }
  if (variant >= 2 && variant <= 4) {
    if (a.nx % 4 != 0) return false;
    int nb = ((a.nx + 255) / 256) * ((a.ny + 3) / 4);
    const void *f = variant == 2 ? (const void *)heat3d_vec_kernel<false, false>
                  : variant == 3 ? (const void *)heat3d_vec_kernel<true, false>
                                 : (const void *)heat3d_vec_kernel<true, true>;
    L.set(f, dim3(xcd_padded_grid(nb)), dim3(64, 4), 0, a);
    return true;
  }
  if (variant != 1) return false;
  int nb = ((a.nx + kDX - 1) / kDX) * ((a.ny + kDY - 1) / kDY);
  L.set((const void *)heat3d_kernel, dim3(xcd_padded_grid(nb)), dim3(kDX, kDY), 0, a);
  return true;
}

// ---------------------------------------------------------------------------
// Many-grid kernel: one launch advances every grid by one step.  The grids'
// 64x4 tiles are numbered consecutively; a block finds its grid by binary
// search over the prefix sums of tiles per grid.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void heat2d_multi_kernel(const MultiArgs a) {
  const int nb = a.block_start[a.G];
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  int lo = 0, hi = a.G - 1;
  while (lo < hi) {            // largest g with block_start[g] <= lb
    const int mid = (lo + hi + 1) >> 1;
    if (a.block_start[mid] <= lb) lo = mid; else hi = mid - 1;
  }
  const GridDesc gd = a.grids[lo];
  const int local = lb - gd.block0;
  const int j = (local % gd.tiles_x) * kMultiBX + threadIdx.x;
  const int i = (local / gd.tiles_x) * kMultiBY + threadIdx.y;
  if (i >= gd.ny || j >= gd.nx) return;
  const size_t nx = (size_t)gd.nx;
  const float *T = a.T + gd.off;
  const int in = i > 0 ? i - 1 : 0;
  const int is = i < gd.ny - 1 ? i + 1 : gd.ny - 1;
  const int jw = j > 0 ? j - 1 : 0;
  const int je = j < gd.nx - 1 ? j + 1 : gd.nx - 1;
  const size_t c = (size_t)i * nx + j;
  const float v = heat_update(T[c], T[(size_t)in * nx + j], T[(size_t)is * nx + j], T[(size_t)i * nx + jw],
                              T[(size_t)i * nx + je], a.P[gd.off + c], a.k);
  a.out[gd.off + c] = v;
}

// Many-grid strip kernel: wave w of a block walks rows i0 .. i0+7 of 64
// consecutive columns (one per lane), keeping the rows above, at and below
// the current one in registers; east / west neighbours come from the
// adjacent lanes, lanes 0 and 63 load the cell beyond the wave (clamped at
// the grid edge).  Same update, same bits as the one-cell kernel.
__global__ __launch_bounds__(256) void heat2d_multi_strip_kernel(const MultiStripArgs a) {
  const int lb = xcd_logical_block(a.nb);
  if (lb >= a.nb) return;
  const GridDesc gd = a.grids[a.block_grid[lb]];
  const int local = lb - gd.block0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nx = gd.nx, ny = gd.ny;
  const int j = (local % gd.tiles_x) * 64 + lane;
  const int i0 = (local / gd.tiles_x) * kStripTileY + wave * kStripRows;
  if (i0 >= ny) return;                       // uniform per wave
  const bool col = j < nx;
  const int jc = col ? j : nx - 1;
  const float *T = a.T + gd.off;
  const float *P = a.P + gd.off;
  float *O = a.out + gd.off;
  float up = T[(size_t)(i0 > 0 ? i0 - 1 : 0) * nx + jc];
  float cur = T[(size_t)i0 * nx + jc];
  const int i1 = min(i0 + kStripRows, ny);
  for (int i = i0; i < i1; ++i) {
    const float down = T[(size_t)(i + 1 < ny ? i + 1 : ny - 1) * nx + jc];
    float wv = lane_west_open(cur);
    float ev = lane_east_open(cur);
    if (lane == 0) wv = jc > 0 ? T[(size_t)i * nx + jc - 1] : cur;
    if (jc >= nx - 1) ev = cur;
    else if (lane == 63) ev = T[(size_t)i * nx + jc + 1];
    const float v = heat_update(cur, up, down, wv, ev, P[(size_t)i * nx + jc], a.k);
    if (col) O[(size_t)i * nx + j] = v;
    up = cur;
    cur = down;
  }
}

// Many-grid temporal blocking (variants 3 and 4): t steps per launch.  Each
// grid is cut into output tiles of (64 - 2t) x (16*NW - 2t) cells; a block
// of NW waves loads its tile grown by t cells on each side (at most 64 x
// 16*NW, clamped to its grid) and advances that region t steps with the
// rows in registers: wave w holds region rows 16w .. 16w+15 of column
// `lane`, east / west neighbours come from the adjacent lanes, north /
// south from the wave's own registers except at its strip ends, which are
// exchanged through LDS (double buffered: one barrier per step).  Cells
// next to a cut halo see a wrong neighbour; that error moves inward one
// cell per step and never reaches the tile, so the result equals t single
// steps bit for bit.  Only a region side that lies on its grid's edge needs
// the clamped neighbour, so the step loop is specialised on which of the
// west, east and south sides do (the north one never needs a select: the
// top row's "row above" starts as the row itself); most regions of a large
// grid take the loop with no clamp at all.
constexpr int kMtRows = 16;                  // region rows per wave

// One step of a region column's 16 rows from `a` to `o` (strip ends read
// from LDS buffer b, written to b^1).  Writing the step into other
// registers than it reads keeps the old row alive as the next row's north
// neighbour without register copies.
template <int NW, bool CW, bool CE, bool CS>
__device__ __forceinline__ void multi_tb_step(const float (&a)[kMtRows], float (&o)[kMtRows],
                                              const float (&pw)[kMtRows], float (*ends)[2][NW][kMtRegionX],
                                              int b, int W, int last, int cx, int w, const HeatCoef &k) {
  const float top = w > 0 ? ends[b][1][w - 1][cx] : a[0];            // old row above
  const float bot = w < NW - 1 ? ends[b][0][w + 1][cx] : a[kMtRows - 1];
#pragma unroll
  for (int i = 0; i < kMtRows; ++i) {
    const float c = a[i];
    const float n = i == 0 ? top : a[i - 1];
    float so = i == kMtRows - 1 ? bot : a[i + 1];
    if (CS && i == last) so = c;
    float ev = lane_east_open(c), wv = lane_west_open(c);
    if (CE && cx >= W - 1) ev = c;
    if (CW && cx == 0) wv = c;
    o[i] = heat_update(c, n, so, wv, ev, pw[i], k);
  }
  ends[b ^ 1][0][w][cx] = o[0];
  ends[b ^ 1][1][w][cx] = o[kMtRows - 1];
  __syncthreads();
}

// t steps, two at a time between two register sets.
template <int NW, bool CW, bool CE, bool CS>
__device__ __forceinline__ void multi_tb_advance(float (&v)[kMtRows], const float (&pw)[kMtRows],
                                                 float (*ends)[2][NW][kMtRegionX], int t, int W, int H,
                                                 int cx, int w, const HeatCoef &k) {
  const int last = H - 1 - kMtRows * w;       // this wave's index of the grid's bottom row (CS)
  float u[kMtRows];
  int s = 0;
  for (; s + 2 <= t; s += 2) {
    multi_tb_step<NW, CW, CE, CS>(v, u, pw, ends, 0, W, last, cx, w, k);
    multi_tb_step<NW, CW, CE, CS>(u, v, pw, ends, 1, W, last, cx, w, k);
  }
  if (s < t) {
    multi_tb_step<NW, CW, CE, CS>(v, u, pw, ends, 0, W, last, cx, w, k);
#pragma unroll
    for (int i = 0; i < kMtRows; ++i) v[i] = u[i];
  }
}

// One temporal-blocking tile of grid `gd` (tile number `local` within the
// grid): load, t steps, store.  ends: the block's LDS strip-end buffers
// [buffer][top, bottom][wave][column].
template <int NW>
__device__ __forceinline__ void region_tb_tile(const GridDesc &gd, int local, const float *__restrict__ Tg,
                                               float *__restrict__ Og, const float *__restrict__ Pg, int t,
                                               const HeatCoef &k, float (*ends)[2][NW][kMtRegionX]) {
  const int tile_x = kMtRegionX - 2 * t, tile_y = kMtRows * NW - 2 * t;
  const int x0 = (local % gd.tiles_x) * tile_x, y0 = (local / gd.tiles_x) * tile_y;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + tile_x + t, gd.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + tile_y + t, gd.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo;
  const int cx = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int r0 = kMtRows * w;
  const int col = cx < W ? cx : W - 1;
  const unsigned nx = (unsigned)gd.nx;
  const size_t base = (size_t)gd.off + (size_t)ry_lo * nx + rx_lo;
  const float *T = Tg + base;
  const float *P = Pg + base;
  float v[kMtRows], pw[kMtRows];
#pragma unroll
  for (int i = 0; i < kMtRows; ++i) {
    const unsigned r = r0 + i < H ? r0 + i : H - 1;
    const unsigned o = r * nx + col;           // < 2^31: a region spans at most 128 rows of a grid
    v[i] = T[o];
    pw[i] = P[o];
  }
  ends[0][0][w][cx] = v[0];
  ends[0][1][w][cx] = v[kMtRows - 1];
  __syncthreads();
  switch ((rx_lo == 0) | (rx_hi == gd.nx) << 1 | (ry_hi == gd.ny) << 2) {
    case 0: multi_tb_advance<NW, false, false, false>(v, pw, ends, t, W, H, cx, w, k); break;
    case 1: multi_tb_advance<NW, true, false, false>(v, pw, ends, t, W, H, cx, w, k); break;
    case 2: multi_tb_advance<NW, false, true, false>(v, pw, ends, t, W, H, cx, w, k); break;
    case 3: multi_tb_advance<NW, true, true, false>(v, pw, ends, t, W, H, cx, w, k); break;
    case 4: multi_tb_advance<NW, false, false, true>(v, pw, ends, t, W, H, cx, w, k); break;
    case 5: multi_tb_advance<NW, true, false, true>(v, pw, ends, t, W, H, cx, w, k); break;
    case 6: multi_tb_advance<NW, false, true, true>(v, pw, ends, t, W, H, cx, w, k); break;
    default: multi_tb_advance<NW, true, true, true>(v, pw, ends, t, W, H, cx, w, k); break;
  }
  const int gx = rx_lo + cx;
  if (cx < W && gx >= x0 && gx < x0 + tile_x) {
    float *O = Og + base;
#pragma unroll
    for (int i = 0; i < kMtRows; ++i) {
      const int gy = ry_lo + r0 + i;
      if (r0 + i < H && gy >= y0 && gy < y0 + tile_y) O[(unsigned)(r0 + i) * nx + cx] = v[i];
    }
  }
}

// The tile of many-grid block lb.
template <int NW>
__device__ __forceinline__ void multi_tb_tile(const MultiTbArgs &a, int lb, float (*ends)[2][NW][kMtRegionX]) {
  const GridDesc gd = a.grids[a.block_grid[lb]];
  region_tb_tile<NW>(gd, lb - gd.block0, a.T, a.out, a.P, a.tdepth, a.k, ends);
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void heat2d_multi_tb_kernel(const MultiTbArgs a) {
  __shared__ float ends[2][2][NW][kMtRegionX];
  const int lb = xcd_logical_block(a.nb);
  if (lb >= a.nb) return;
  multi_tb_tile<NW>(a, lb, ends);
}

// One large grid with the same region tiles (variants 18 and 19): the
// tiling of a single grid of the many-grid kernel, with no tables.  Honours
// the run flag of the tile kernels.
template <int NW>
__global__ __launch_bounds__(64 * NW) void heat2d_region_tb_kernel(const Heat2DArgs a) {
  __shared__ float ends[2][2][NW][kMtRegionX];
  if (a.flag && *a.flag == 0) return;
  const int t = a.tdepth;
  const int tiles_x = (a.nx + multi_tb_tile_x(0, t) - 1) / multi_tb_tile_x(0, t);
  const int tiles_y = (a.ny + kMtRows * NW - 2 * t - 1) / (kMtRows * NW - 2 * t);
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const GridDesc gd{0, a.ny, a.nx, tiles_x, 0};
  region_tb_tile<NW>(gd, lb, a.T, a.out, a.P, t, a.k, ends);
}

// Regions two columns per lane wide (variants 20 and 21): 128 columns x
// 16*NW rows, lane cx holding region columns 2cx and 2cx+1 of 16 rows.  The
// wider region recomputes fewer halo cells per output cell (at t = 6,
// 128 x 128 regions around 116 x 116 tiles instead of 64 x 128 around
// 52 x 116), and the two columns of a lane are each other's east / west
// neighbours, so a cell pair needs two lane shifts instead of four.  The
// clamps and the strip-end exchange are those of the one-column regions.
constexpr int kRg2X = 128;

// t steps of a two-column region (columns 2cx, 2cx+1 of 16 rows in v0,
// v1).  Strip ends go through LDS with region column c at LDS column
// (c & 1) * 64 + c / 2, so that a wave's accesses are to consecutive
// words.  Unlike the one-column regions the steps update the rows in place:
// a second register set would take the kernel past 128 VGPRs and halve the
// waves per SIMD.
template <int NW, bool CW, bool CE, bool CS>
__device__ __forceinline__ void region2_advance(float (&v0)[kMtRows], float (&v1)[kMtRows],
                                                const float (&p0)[kMtRows], const float (&p1)[kMtRows],
                                                float (*ends)[2][NW][kRg2X], int t, int W, int H, int cx,
                                                int w, const HeatCoef &k) {
  const int last = H - 1 - kMtRows * w;
  const int c0 = 2 * cx, c1 = 2 * cx + 1;
  int b = 0;
  for (int s = 0; s < t; ++s) {
    float prev0 = w > 0 ? ends[b][1][w - 1][cx] : v0[0];
    float prev1 = w > 0 ? ends[b][1][w - 1][64 + cx] : v1[0];
    const float bot0 = w < NW - 1 ? ends[b][0][w + 1][cx] : v0[kMtRows - 1];
    const float bot1 = w < NW - 1 ? ends[b][0][w + 1][64 + cx] : v1[kMtRows - 1];
#pragma unroll
    for (int i = 0; i < kMtRows; ++i) {
      const float a0 = v0[i], a1 = v1[i];
      float s0 = i == kMtRows - 1 ? bot0 : v0[i + 1];
      float s1 = i == kMtRows - 1 ? bot1 : v1[i + 1];
      if (CS && i == last) {
        s0 = a0;
        s1 = a1;
      }
      float w0 = lane_west_open(a1), e1 = lane_east_open(a0);
      float e0 = a1;
      if (CW && cx == 0) w0 = a0;
      if (CE && c0 >= W - 1) e0 = a0;
      if (CE && c1 >= W - 1) e1 = a1;
      const float n0 = prev0, n1 = prev1;
      prev0 = a0;
      prev1 = a1;
      v0[i] = heat_update(a0, n0, s0, w0, e0, p0[i], k);
      v1[i] = heat_update(a1, n1, s1, a0, e1, p1[i], k);
    }
    b ^= 1;
    ends[b][0][w][cx] = v0[0];
    ends[b][0][w][64 + cx] = v1[0];
    ends[b][1][w][cx] = v0[kMtRows - 1];
    ends[b][1][w][64 + cx] = v1[kMtRows - 1];
    __syncthreads();
  }
}

template <int NW>
__device__ __forceinline__ void region2_tile(const GridDesc &gd, int local, const float *__restrict__ Tg,
                                             float *__restrict__ Og, const float *__restrict__ Pg, int t,
                                             const HeatCoef &k, float (*ends)[2][NW][kRg2X]) {
  const int tile_x = kRg2X - 2 * t, tile_y = kMtRows * NW - 2 * t;
  const int x0 = (local % gd.tiles_x) * tile_x, y0 = (local / gd.tiles_x) * tile_y;
  const int rx_lo = max(x0 - t, 0), rx_hi = min(x0 + tile_x + t, gd.nx);
  const int ry_lo = max(y0 - t, 0), ry_hi = min(y0 + tile_y + t, gd.ny);
  const int W = rx_hi - rx_lo, H = ry_hi - ry_lo;
  const int cx = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = kMtRows * w;
  const int col0 = 2 * cx < W ? 2 * cx : W - 1;
  const int col1 = 2 * cx + 1 < W ? 2 * cx + 1 : W - 1;
  const unsigned nx = (unsigned)gd.nx;
  const size_t base = (size_t)gd.off + (size_t)ry_lo * nx + rx_lo;
  const float *T = Tg + base;
  const float *P = Pg + base;
  float v0[kMtRows], v1[kMtRows], p0[kMtRows], p1[kMtRows];
#pragma unroll
  for (int i = 0; i < kMtRows; ++i) {
    const unsigned r = r0 + i < H ? r0 + i : H - 1;
    v0[i] = T[r * nx + col0];                  // < 2^31: a region spans at most 128 rows
    v1[i] = T[r * nx + col1];
    p0[i] = P[r * nx + col0];
    p1[i] = P[r * nx + col1];
  }
  ends[0][0][w][cx] = v0[0];
  ends[0][0][w][64 + cx] = v1[0];
  ends[0][1][w][cx] = v0[kMtRows - 1];
  ends[0][1][w][64 + cx] = v1[kMtRows - 1];
  __syncthreads();
  switch ((rx_lo == 0) | (rx_hi == gd.nx) << 1 | (ry_hi == gd.ny) << 2) {
    case 0: region2_advance<NW, false, false, false>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 1: region2_advance<NW, true, false, false>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 2: region2_advance<NW, false, true, false>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 3: region2_advance<NW, true, true, false>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 4: region2_advance<NW, false, false, true>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 5: region2_advance<NW, true, false, true>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    case 6: region2_advance<NW, false, true, true>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
    default: region2_advance<NW, true, true, true>(v0, v1, p0, p1, ends, t, W, H, cx, w, k); break;
  }
  float *O = Og + base;
#pragma unroll
  for (int i = 0; i < kMtRows; ++i) {
    const int gy = ry_lo + r0 + i;
    if (r0 + i < H && gy >= y0 && gy < y0 + tile_y) {
      const int g0 = rx_lo + 2 * cx;
      if (2 * cx < W && g0 >= x0 && g0 < x0 + tile_x) O[(unsigned)(r0 + i) * nx + 2 * cx] = v0[i];
      if (2 * cx + 1 < W && g0 + 1 >= x0 && g0 + 1 < x0 + tile_x) O[(unsigned)(r0 + i) * nx + 2 * cx + 1] = v1[i];
    }
  }
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void heat2d_region2_tb_kernel(const Heat2DArgs a) {
  __shared__ float ends[2][2][NW][kRg2X];
  if (a.flag && *a.flag == 0) return;
  const int t = a.tdepth;
  const int tiles_x = (a.nx + kRg2X - 2 * t - 1) / (kRg2X - 2 * t);
  const int tiles_y = (a.ny + kMtRows * NW - 2 * t - 1) / (kMtRows * NW - 2 * t);
  const int nb = tiles_x * tiles_y;
  const int lb = xcd_logical_block(nb);
  if (lb >= nb) return;
  const GridDesc gd{0, a.ny, a.nx, tiles_x, 0};
  region2_tile<NW>(gd, lb, a.T, a.out, a.P, t, a.k, ends);
}

// Many-grid temporal blocking over regions two columns per lane wide
// (variants 5 and 6).
template <int NW>
__global__ __launch_bounds__(64 * NW) void heat2d_multi_tb2_kernel(const MultiTbArgs a) {
  __shared__ float ends[2][2][NW][kRg2X];
  const int lb = xcd_logical_block(a.nb);
  if (lb >= a.nb) return;
  const GridDesc gd = a.grids[a.block_grid[lb]];
  region2_tile<NW>(gd, lb - gd.block0, a.T, a.out, a.P, a.tdepth, a.k, ends);
}

// variant 18: 64 x 64 regions (4 waves), 19: 64 x 128 (8 waves); two
// columns per lane: 20: 128 x 64, 21: 128 x 128
bool make_heat2d_region(Launch &L, const Heat2DArgs &a, int variant) {
  if (a.tdepth < 1 || a.tdepth > kMtMaxDepth) return false;
  const int nw = variant == 19 || variant == 21 ? 8 : 4;
  const int tx = variant >= 20 ? kRg2X - 2 * a.tdepth : multi_tb_tile_x(0, a.tdepth);
  const long long tiles_x = (a.nx + tx - 1) / tx;
  const long long tiles_y = (a.ny + kMtRows * nw - 2 * a.tdepth - 1) / (kMtRows * nw - 2 * a.tdepth);
  if (tiles_x * tiles_y > (1LL << 30)) return false;
  const dim3 grid(xcd_padded_grid((int)(tiles_x * tiles_y)));
  if (variant == 18) L.set((const void *)heat2d_region_tb_kernel<4>, grid, dim3(256), 0, a);
  else if (variant == 19) L.set((const void *)heat2d_region_tb_kernel<8>, grid, dim3(512), 0, a);
  else if (variant == 20) L.set((const void *)heat2d_region2_tb_kernel<4>, grid, dim3(256), 0, a);
  else if (variant == 21) L.set((const void *)heat2d_region2_tb_kernel<8>, grid, dim3(512), 0, a);
  else return false;
  return true;
}

// ---------------------------------------------------------------------------
// Persistent many-grid kernel: one cooperative launch advances every grid by
// n steps, as nfull super-steps of t steps and one of rem steps, each a pass
// of the temporal-blocking tiles over the whole set of grids followed by a
// grid-wide barrier (the buffers then swap).  The blocks of XCD x take the
// x-th eighth of the tile list, so neighbouring tiles share an L2.
// ---------------------------------------------------------------------------

// Grid-wide barrier of a cooperative launch (every block resident).  Each
// wave first waits until its own stores have reached the L2 (vmcnt 0; on
// gfx9 this counter covers stores), so after the block barrier one device-
// scope release by thread 0 writes the whole block's results back from the
// XCD's L2.  Arrival is counted in two levels so that no counter takes more
// than a few dozen atomics per barrier: a block counts in at the counter of
// its group (blockIdx mod kBarGroups), the group's last block counts in at
// the top counter, and the last group's block moves the generation on.  The
// other blocks poll the generation; the device-scope acquire of thread 0
// then invalidates the CU's L1 and the XCD's L2 for every wave of the block.
// A wait longer than spin_limit polls raises the error flag, after which no
// block waits any more, so the grid always drains (the host then reports
// the run as failed).
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned nblocks, unsigned &gen, unsigned spin_limit) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned groups = nblocks < kBarGroups ? nblocks : kBarGroups;
    const unsigned g = blockIdx.x % groups;
    const unsigned members = (nblocks - g + groups - 1) / groups;   // blocks of group g
    unsigned *sub = bar + kBarStride * (1 + g);
    bool released = false;
    if (__hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");           // the group's results
      __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == groups - 1) {
        __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bar[1], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        released = true;
      }
    }
    if (!released) {
      unsigned spins = 0;
      // relaxed polls: an acquiring load would invalidate the XCD's L2 on
      // every poll, under the blocks that are still working
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen &&
             __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        if (++spins > spin_limit) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  ++gen;
  __syncthreads();
}

__global__ __launch_bounds__(256) void heat2d_multi_persistent_kernel(const MultiPersistArgs a) {
  __shared__ float ends[2][2][4][kMtRegionX];
  float *src = a.T0, *dst = a.T1;
  unsigned gen = 0;
  const int nsuper = a.nfull + (a.rem > 0 ? 1 : 0);
  const int per_xcd = gridDim.x / kXcds, x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  for (int s = 0; s < nsuper; ++s) {
    const int d = s < a.nfull ? a.tdepth : a.rem;
    const MultiTbArgs ta{src, dst, a.P, a.grids + (size_t)(d - 1) * a.G, a.block_grid + a.tb_start[d - 1],
                         a.tb_start[d] - a.tb_start[d - 1], d, a.k};
    const int per = (ta.nb + kXcds - 1) / kXcds;
    const int hi = min((x + 1) * per, ta.nb);
    for (int lb = x * per + i; lb < hi; lb += per_xcd) multi_tb_tile<4>(ta, lb, ends);
    grid_barrier(a.bar, gridDim.x, gen, a.spin_limit);
    float *tmp = src;
    src = dst;
    dst = tmp;
  }
}

const void *multi_persistent_fn() { return (const void *)heat2d_multi_persistent_kernel; }

void make_multi_tb(Launch &L, const MultiTbArgs &a, int shape) {
  const dim3 grid(xcd_padded_grid(a.nb));
  if (shape == 0) L.set((const void *)heat2d_multi_tb_kernel<4>, grid, dim3(256), 0, a);
  else if (shape == 1) L.set((const void *)heat2d_multi_tb_kernel<8>, grid, dim3(512), 0, a);
  else if (shape == 2) L.set((const void *)heat2d_multi_tb2_kernel<4>, grid, dim3(256), 0, a);
  else L.set((const void *)heat2d_multi_tb2_kernel<8>, grid, dim3(512), 0, a);
}

void make_multi_strip(Launch &L, const MultiStripArgs &a) {
  L.set((const void *)heat2d_multi_strip_kernel, dim3(xcd_padded_grid(a.nb)), dim3(256), 0, a);
}

void make_multi(Launch &L, const MultiArgs &a, int total_blocks) {
  L.set((const void *)heat2d_multi_kernel, dim3(xcd_padded_grid(total_blocks)), dim3(kMultiBX, kMultiBY), 0, a);
}

}  // namespace kb
