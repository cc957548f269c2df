// libkbatch C ABI: problem objects, the per-launch driver, the graph
// builders (explicit kernel nodes, stream capture), graph replay with loop
// peeling, timing, reads, writes and reductions.
//
// The method (Sec. III-A): an iterative application runs `n` iterations of
// a fixed sequence of K kernels.  The baseline enqueues every kernel of
// every iteration separately (Listings 1-2).  The batched form unrolls an
// iteration batch of b iterations into one static graph -- a linear chain of
// K*b kernel nodes, each depending on the previous one (Listing 3) --
// instantiates and uploads it once, and launches it n/b times.  Sec. VI names
// loop peeling for n not divisible by b; here the n mod b leftover
// iterations run per launch after the replays.
//
// Kernel arguments are baked into graph nodes.  For the ping-pong stencils
// the input buffer alternates each iteration, so a batch graph is specific
// to the buffer parity it starts from; with odd b successive replays
// alternate between two graphs.  State that must change with the absolute
// step (the FDTD source time) lives on the device instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "kb_internal.h"

using namespace kb;

namespace {

thread_local std::string g_err;

}  // namespace

int kb::kb_set_error(int code, const char *msg) {
  g_err = msg;
  return code;
}

namespace {

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(KB_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kGCap = 4096;           // FDTD source table capacity (steps)
constexpr int64_t kDefaultProbe = 16384;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t off = total;
    total = align_up(total + bytes);
    return off;
  }
};

bool heat_shape_ok(int64_t v) { return v >= 1 && v <= (int64_t)1 << 20; }

// FDTD row pitch: N+1 nodes rounded up to a multiple of 4 floats (16 bytes).
int64_t fdtd_pitch(int64_t N) { return (N + 1 + 3) / 4 * 4; }

// Workspace offsets of every buffer of a problem.  Returns false on a bad
// shape.  Offsets are written to off[] in the order documented per problem.
bool layout(int problem, const int64_t *shape, int ndim, Layout &L, size_t *off) {
  if (!shape || ndim < 1) return false;
  const size_t red = 2 * (size_t)reduce_max_blocks() * sizeof(double);
  // reduction partials, result, and the log of in-chain reductions
  auto common = [&]() {
    off[3] = L.add(red); off[4] = L.add(64);
    off[16] = L.add((size_t)kRedLogCap * 4 * sizeof(double)); off[17] = L.add(8);
  };
  switch (problem) {
    case KB_HEAT2D: {
      if (ndim != 2 || !heat_shape_ok(shape[0]) || !heat_shape_ok(shape[1])) return false;
      const int64_t n = shape[0] * shape[1];
      if (n > ((int64_t)1 << 31) - 1) return false;
      off[0] = L.add(n * 4); off[1] = L.add(n * 4); off[2] = L.add(n * 4);
      common();
      return true;
    }
    case KB_HEAT3D: {
      if (ndim != 3 || !heat_shape_ok(shape[0]) || !heat_shape_ok(shape[1]) || !heat_shape_ok(shape[2])) return false;
      const int64_t plane = shape[1] * shape[2];
      const int64_t n = shape[0] * plane;
      if (n > ((int64_t)1 << 31) - 1) return false;
      off[0] = L.add(n * 4); off[1] = L.add(n * 4); off[2] = L.add(plane * 4);
      common();
      return true;
    }
    case KB_SKELETON: {
      if (ndim != 1 || shape[0] < 1 || shape[0] > ((int64_t)1 << 31) - 1) return false;
      off[0] = L.add(shape[0] * 4);
      common();
      return true;
    }
    case KB_FDTD3D: {
      if (ndim < 1 || ndim > 2 || shape[0] < 4 || shape[0] > 1024) return false;
      const int64_t pcap = ndim == 2 ? shape[1] : kDefaultProbe;
      if (pcap < 0 || pcap > ((int64_t)1 << 28)) return false;
      const int64_t M = shape[0] + 1;
      // two sets of the six fields
      for (int f = 0; f < 6; ++f) off[5 + f] = L.add(M * M * fdtd_pitch(shape[0]) * 4);
      for (int f = 0; f < 6; ++f) off[23 + f] = L.add(M * M * fdtd_pitch(shape[0]) * 4);
      off[11] = L.add(kGCap * 4);
      off[12] = L.add((pcap > 0 ? pcap : 1) * 4);
      off[13] = L.add(16);              // step counter, finished-block counter
      common();
      return true;
    }
    case KB_HEAT2D_MULTI: {
      if (ndim < 3) return false;
      const int64_t G = shape[0];
      if (G < 1 || G > 65536 || ndim != 1 + 2 * G) return false;
      int64_t total = 0;
      for (int64_t g = 0; g < G; ++g) {
        if (!heat_shape_ok(shape[1 + 2 * g]) || !heat_shape_ok(shape[2 + 2 * g])) return false;
        total += shape[1 + 2 * g] * shape[2 + 2 * g];
      }
      if (total > ((int64_t)1 << 31) - 1) return false;
      off[0] = L.add(total * 4); off[1] = L.add(total * 4); off[2] = L.add(total * 4);
      off[14] = L.add(G * sizeof(GridDesc)); off[15] = L.add((G + 1) * sizeof(int));
      int64_t nb2 = 0;
      for (int64_t g = 0; g < G; ++g)
        nb2 += ((shape[2 + 2 * g] + 63) / 64) * ((shape[1 + 2 * g] + kStripTileY - 1) / kStripTileY);
      if (nb2 > ((int64_t)1 << 30)) return false;
      off[18] = L.add(G * sizeof(GridDesc)); off[19] = L.add(nb2 * sizeof(int));
      // temporal-blocking tilings, one per (region shape, depth)
      int64_t nbt = 0;
      for (int sh = 0; sh < kMtShapes; ++sh)
        for (int t = 1; t <= kMtMaxDepth; ++t) {
          const int64_t tx = multi_tb_tile_x(sh, t), ty = multi_tb_tile_y(sh, t);
          for (int64_t g = 0; g < G; ++g)
            nbt += ((shape[2 + 2 * g] + tx - 1) / tx) * ((shape[1 + 2 * g] + ty - 1) / ty);
        }
      if (nbt > ((int64_t)1 << 30)) return false;
      off[20] = L.add(kMtTilings * G * sizeof(GridDesc)); off[21] = L.add(nbt * sizeof(int));
      off[22] = L.add(kBarWords * sizeof(unsigned));   // persistent kernel's barrier
      common();
      return true;
    }
    case KB_HEAT2D_SURROGATE: {
      const size_t sg = sg_workspace_bytes(shape, ndim);
      if (!sg) return false;
      L.total = sg;
      off[3] = L.add(red); off[4] = L.add(64);
      return true;
    }
    default:
      return false;
  }
}

bool pingpong(const kb_problem *h) {
  return h->kind == KB_HEAT2D || h->kind == KB_HEAT3D || h->kind == KB_HEAT2D_MULTI ||
         h->kind == KB_HEAT2D_SURROGATE;
}

// FDTD kernel variant: the fused H + E step unless another is chosen, with
// streaming stores once the two field sets outgrow the 256 MB last-level
// cache (they then go to HBM anyway; keeping them out of L2 leaves it to the
// neighbouring rows and planes being read), plain stores below that (where
// the next step reads them back from that cache).
int fdtd_variant(const kb_problem *h) {
  if (h->tile != 0) return h->tile;
  const double sets = 12.0 * (h->N + 1) * (h->N + 1) * h->pitch * 4;
  return sets > 256.0 * (1 << 20) ? 7 : 5;
}

// Kernels per FDTD iteration: separate H, E and source (variants < 5); one
// whole-row launch of two or three steps (9, 10 at depth 2 or 3 up to
// N = 256); else a step kernel (fused, or the two-step tiles) and the
// source or step advance.
int fdtd_kernels_per_iter(const kb_problem *h) {
  const int v = fdtd_variant(h);
  if (v < 5) return 3;
  return v >= 9 && (h->tdepth == 2 || h->tdepth == 3) && h->N <= 256 ? 1 : 2;
}

// Does an iteration move the state to the other buffer set?  The stencils'
// ping-pong buffers, and the FDTD fields under the fused step.
bool alternates(const kb_problem *h) {
  return pingpong(h) || (h->kind == KB_FDTD3D && fdtd_variant(h) >= 5);
}

// Kernel variant in use: the option, or the default for the shape (vector
// rows when every row is 16-byte aligned, else one thread per cell).
// Measured on MI355X: the vector kernels win once a plane has about a
// million cells; below that the one-thread-per-cell kernels have more waves
// in flight and are faster.
int heat2d_variant(const kb_problem *h) {
  if (h->tile != 0) return h->tile;
  return (h->nx % 4 == 0 && h->ny * h->nx >= (1 << 20)) ? 13 : 1;
}
int heat3d_variant(const kb_problem *h) {
  if (h->tile != 0) return h->tile;
  return (h->nx % 4 == 0 && h->ny * h->nx >= (1 << 20)) ? 9 : 1;
}
bool heat2d_is_tile(int v) { return (v >= 2 && v <= 7) || (v >= 15 && v <= 23); }   // temporal blocking

// Many-grid variants 3 to 6 (and the default, 3) block in time.
bool multi_is_tb(const kb_problem *h) { return h->tile == 0 || (h->tile >= 3 && h->tile <= 6); }
// Their region shapes: variant 3 -> 0, 4 -> 1, 5 -> 2, 6 -> 3.
int multi_tb_shape(const kb_problem *h) { return h->tile >= 4 ? h->tile - 3 : 0; }

// Temporal depth of one iteration.
int iter_depth(const kb_problem *h) {
  if (h->kind == KB_HEAT2D_SURROGATE) return sg_iter_depth(h);
  if (h->kind == KB_HEAT3D && (heat3d_variant(h) == 5 || heat3d_variant(h) == 11)) return h->tdepth;
  if (h->kind == KB_HEAT2D_MULTI && multi_is_tb(h)) return h->tdepth;
  if (h->kind == KB_FDTD3D && fdtd_variant(h) >= 8) return h->tdepth;
  return (h->kind == KB_HEAT2D && heat2d_is_tile(heat2d_variant(h))) ? h->tdepth : 1;
}

// The two launches of an in-chain reduction of the state after an
// iteration that started from parity `cur`: the sum of T (heat problems),
// of x (skeleton), or E.E and H.H (FDTD).
int fill_reduce(const kb_problem *h, int cur, Launch *L) {
  RedLogArgs a{};
  if (pingpong(h)) {
    const float *f[1] = {h->Tbuf[1 - cur]};
    const long long n = h->kind == KB_HEAT2D_MULTI ? h->total_cells : h->nz * h->ny * h->nx;
    a = reduce_log_args(f, 1, 1, 0, n, h->partials, h->redlog, h->redcount, h->red_every);
  } else if (h->kind == KB_SKELETON) {
    const float *f[1] = {h->x};
    a = reduce_log_args(f, 1, 1, 0, h->n, h->partials, h->redlog, h->redcount, h->red_every);
  } else {
    // padded FDTD arrays: the padding columns hold zeros and add nothing;
    // the set the iteration wrote: the other one after a fused step
    const long long n = (long long)(h->N + 1) * (h->N + 1) * h->pitch;
    const float *F[6];
    for (int f = 0; f < 6; ++f) F[f] = h->F[alternates(h) ? 1 - cur : cur][f];
    a = reduce_log_args(F, 6, 2, 1, n, h->partials, h->redlog, h->redcount, h->red_every);
  }
  make_reduce_log(L[0], L[1], a);
  return 2;
}

// Does the iteration that starts `steps_before` steps after the reduction
// option was set end on a reduction point?
bool reduce_due(const kb_problem *h, int64_t steps_before, int depth) {
  return h->red_every > 0 && (steps_before + depth) % h->red_every == 0;
}

int fill_iter_kernels(const kb_problem *h, int cur, int depth, Launch *L);

// Fill the launch descriptors of one iteration that starts from buffer
// parity `cur` and advances `depth` steps, plus the reduction after it when
// reduce_after is set.
int fill_iter(const kb_problem *h, int cur, int depth, Launch *L, bool reduce_after) {
  const int k = fill_iter_kernels(h, cur, depth, L);
  if (k < 0 || !reduce_after) return k;
  return k + fill_reduce(h, cur, L + k);
}

int fill_iter_kernels(const kb_problem *h, int cur, int depth, Launch *L) {
  switch (h->kind) {
    case KB_HEAT2D: {
      Heat2DArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, (int)h->ny, (int)h->nx, h->hk, depth};
      const int v = heat2d_variant(h);
      if (v == 1) {
        make_heat2d_direct(L[0], a);
        return 1;
      }
      if (v >= 22) return make_heat2d_strip(L[0], a, v) ? 1 : -1;
      if (v >= 18) return make_heat2d_region(L[0], a, v) ? 1 : -1;
      if (v >= 15) return make_heat2d_strip(L[0], a, v) ? 1 : -1;
      if (heat2d_is_tile(v)) return make_heat2d_tile(L[0], a, v) ? 1 : -1;
      return make_heat2d_vec(L[0], a, v) ? 1 : -1;
    }
    case KB_HEAT3D: {
      Heat3DArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, (int)h->nz, (int)h->ny, (int)h->nx, h->hk, depth};
      return make_heat3d(L[0], a, heat3d_variant(h)) ? 1 : -1;
    }
    case KB_HEAT2D_SURROGATE: {
      if (depth == sg_iter_depth(h)) return sg_fill_iter(h, cur, L);
      // leftover steps: plain single steps
      Heat2DArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, (int)h->ny, (int)h->nx, h->hk, 1};
      make_heat2d_direct(L[0], a);
      return 1;
    }
    case KB_HEAT2D_MULTI: {
      if (h->tile == 1) {
        MultiArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, h->grids_d, h->block_start_d, h->G, h->hk};
        make_multi(L[0], a, h->total_blocks);
      } else if (multi_is_tb(h)) {
        if (depth < 1 || depth > kMtMaxDepth) return -1;
        const int sh = multi_tb_shape(h), q = multi_tb_index(sh, depth);
        MultiTbArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, h->grids_tb_d + (size_t)q * h->G,
                      h->block_grid_tb_d + h->tb_start[q], h->tb_start[q + 1] - h->tb_start[q], depth, h->hk};
        make_multi_tb(L[0], a, sh);
      } else {
        MultiStripArgs a{h->Tbuf[cur], h->Tbuf[1 - cur], h->P, h->grids2_d, h->block_grid_d, h->total_blocks2, h->hk};
        make_multi_strip(L[0], a);
      }
      return 1;
    }
    case KB_SKELETON: {
      for (int k = 0; k < h->K; ++k) {
        SkelArgs a{h->x, (long long)h->n, h->a[k], h->b[k]};
        make_skeleton(L[k], a, h->tile == 0 ? 1 : h->tile);
      }
      return h->K;
    }
    case KB_FDTD3D: {
      float *const *A = h->F[cur];
      const int v = fdtd_variant(h);
      if (v >= 5) {
        float *const *B = h->F[1 - cur];
        // variant 8: two steps per launch (depth 2; streaming stores as 7
        // once the sets outgrow the last-level cache), its single steps the
        // fused step
        const bool nt8 = 12.0 * (h->N + 1) * (h->N + 1) * h->pitch * 4 > 256.0 * (1 << 20);
        if (v >= 8 && (depth == 2 || depth == 3)) {
          FdtdTbArgs t{};
          t.Ex = A[0]; t.Ey = A[1]; t.Ez = A[2]; t.Hx = A[3]; t.Hy = A[4]; t.Hz = A[5];
          t.oEx = B[0]; t.oEy = B[1]; t.oEz = B[2]; t.oHx = B[3]; t.oHy = B[4]; t.oHz = B[5];
          t.N = h->N; t.P = h->pitch; t.dt = h->dt;
          t.si = h->src_ijk[0]; t.sj = h->src_ijk[1]; t.sk = h->src_ijk[2];
          t.g = h->g; t.glen = h->glen; t.probe = h->probe; t.pcap = h->pcap; t.step = h->step;
          // variants 9, 10: whole rows up to N = 256 (above that, as 8);
          // three steps per launch only with whole rows
          if (v >= 9 && h->N <= 256) {
            t.step_w = h->step;
            t.done = h->done;
            if (depth == 3) {
              t.fs = reinterpret_cast<const char *>(A[1]) - reinterpret_cast<const char *>(A[0]);
              return make_fdtd_tb3_rows(L[0], t, nt8) ? 1 : -1;
            }
            return make_fdtd_tb2_rows(L[0], t, nt8, v - 9) ? 1 : -1;
          }
          if (depth == 3 || !make_fdtd_tb2(L[0], t, nt8)) return -1;
          make_fdtd_step_add(L[1], h->step, 2);
          return 2;
        }
        if (v >= 8 && depth != 1) return -1;
        FdtdFusedArgs f{A[0], A[1], A[2], A[3], A[4], A[5], B[0], B[1], B[2], B[3], B[4], B[5],
                        h->N, h->pitch, h->dt};
        // variant 5: one plane per thread; 6: 8 planes; 7: one plane, streaming stores
        if (!make_fdtd_fused(L[0], f, v == 6 ? 8 : 1, v == 7 || (v >= 8 && nt8))) return -1;
        SrcArgs s{B[2], h->src, h->g, h->glen, h->probe, h->pcap, h->step};
        make_fdtd_src(L[1], s);
        return 2;
      }
      FdtdArgs f{A[0], A[1], A[2], A[3], A[4], A[5], h->N, h->pitch, h->dt};
      if (!make_fdtd_h(L[0], f, v) || !make_fdtd_e(L[1], f, v)) return -1;
      SrcArgs s{A[2], h->src, h->g, h->glen, h->probe, h->pcap, h->step};
      make_fdtd_src(L[2], s);
      return 3;
    }
  }
  return -1;
}

constexpr int kMaxK = 16;

// Enqueue one iteration per launch on stream s; returns a KB status.
int launch_iter(kb_problem *h, int depth, hipStream_t s) {
  Launch L[kMaxK];
  const int k = fill_iter(h, h->cur, depth, L, reduce_due(h, h->step_count, depth));
  if (k < 0) return fail(KB_EINVAL, "invalid kernel variant %d / depth %d", h->tile, depth);
  h->step_count += depth;
  for (int q = 0; q < k; ++q) {
    HIPCHK(hipLaunchKernel(L[q].func, L[q].grid, L[q].block, L[q].params(), L[q].lds, s));
  }
  if (alternates(h)) h->cur ^= 1;
  return KB_OK;
}

void clear_cache(kb_problem *h) {
  for (auto &kv : h->cache_map) (void)hipGraphExecDestroy(kv.second);
  h->cache_map.clear();
}

// Record the graph of b iterations starting from buffer parity `parity`,
// `phase` steps after a reduction point (Listing 3, "Building"): explicit
// kernel nodes or stream capture of the per-launch loop.
int make_graph(kb_problem *h, int64_t b, int depth, int parity, int64_t phase, hipGraph_t *out) {
  hipGraph_t g = nullptr;
  const int saved = h->cur;
  const int64_t saved_steps = h->step_count;
  if (h->builder == 0) {
    HIPCHK(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    int c = parity;
    Launch L[kMaxK];
    for (int64_t j = 0; j < b; ++j) {
      const int k = fill_iter(h, c, depth, L, reduce_due(h, phase + j * depth, depth));
      if (k < 0) { (void)hipGraphDestroy(g); return fail(KB_EINVAL, "invalid kernel variant"); }
      for (int q = 0; q < k; ++q) {
        hipKernelNodeParams np{};
        np.func = const_cast<void *>(L[q].func);
        np.gridDim = L[q].grid;
        np.blockDim = L[q].block;
        np.sharedMemBytes = L[q].lds;
        np.kernelParams = L[q].params();
        np.extra = nullptr;
        hipGraphNode_t node = nullptr;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
        if (e != hipSuccess) {
          (void)hipGraphDestroy(g);
          return fail(KB_EHIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
        }
        prev = node;
      }
      if (alternates(h)) c ^= 1;
    }
  } else {
    HIPCHK(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    h->cur = parity;
    h->step_count = phase;
    int rc = KB_OK;
    for (int64_t j = 0; j < b && rc == KB_OK; ++j) rc = launch_iter(h, depth, h->capture_stream);
    hipError_t e = hipStreamEndCapture(h->capture_stream, &g);
    h->cur = saved;
    h->step_count = saved_steps;
    if (rc != KB_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(KB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  *out = g;
  return KB_OK;
}

// Build, instantiate and upload one batch graph.
int build_graph(kb_problem *h, int64_t b, int depth, int parity, int64_t phase, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  const int rc = make_graph(h, b, depth, parity, phase, &g);
  if (rc != KB_OK) return rc;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiateWithFlags(&exec, g, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(KB_EHIP, "hipGraphInstantiateWithFlags: %s", hipGetErrorString(e));
  e = hipGraphUpload(exec, h->stream);
  if (e != hipSuccess) { (void)hipGraphExecDestroy(exec); return fail(KB_EHIP, "hipGraphUpload: %s", hipGetErrorString(e)); }
  *out = exec;
  return KB_OK;
}

// Kernel arguments baked into the nodes changed (skeleton coefficients):
// refit every cached executable graph in place (record the graph again
// with the new arguments, hipGraphExecUpdate: same topology, new node
// parameters, no instantiation) or, where that is refused, drop it.
// Returns the number of graphs updated.
int64_t update_cached(kb_problem *h) {
  int64_t updated = 0;
  for (auto it = h->cache_map.begin(); it != h->cache_map.end();) {
    const auto &k = it->first;
    hipGraph_t g = nullptr;
    bool ok = make_graph(h, std::get<0>(k), std::get<1>(k), std::get<3>(k), std::get<4>(k), &g) == KB_OK;
    if (ok) {
      hipGraphNode_t err_node = nullptr;
      hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
      ok = hipGraphExecUpdate(it->second, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
      (void)hipGraphDestroy(g);
    }
    if (ok) {
      ++updated;
      ++it;
    } else {
      (void)hipGraphExecDestroy(it->second);
      it = h->cache_map.erase(it);
    }
  }
  g_err.clear();
  return updated;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int enqueue_init(kb_problem *h, float *dst, long long n, uint64_t seed, uint64_t tag, uint64_t offset, double lo,
                 double hi) {
  if (n <= 0) return KB_OK;
  Launch L;
  InitArgs a{dst, n, seed, tag, offset, lo, hi - lo};
  make_init(L, a);
  HIPCHK(hipLaunchKernel(L.func, L.grid, L.block, L.params(), 0, h->stream));
  return KB_OK;
}

// Device location and user-visible size of a field.  *host_vec: the field
// lives in host memory of the handle.  *rows/*pitch: > 0 for the FDTD fields,
// whose rows of N+1 floats are stored with a pitch of h->pitch floats on
// the device (the caller sees them dense).
bool field_info(const kb_problem *h, int field, float **dev, size_t *bytes, bool *host_vec, size_t *rows,
                size_t *pitch) {
  *host_vec = false;
  *rows = 0;
  *pitch = 0;
  switch (field) {
    case KB_F_T:
      if (!pingpong(h)) return false;
      *dev = h->Tbuf[h->cur];
      *bytes = (h->kind == KB_HEAT2D_MULTI ? h->total_cells : h->nz * h->ny * h->nx) * 4;
      return true;
    case KB_F_P:
      if (!pingpong(h)) return false;
      *dev = h->P;
      *bytes = (h->kind == KB_HEAT2D_MULTI ? h->total_cells : h->ny * h->nx) * 4;
      return true;
    case KB_F_X:
      if (h->kind != KB_SKELETON) return false;
      *dev = h->x; *bytes = h->n * 4; return true;
    case KB_F_A: case KB_F_B:
      if (h->kind != KB_SKELETON) return false;
      *dev = nullptr; *bytes = h->K * 4; *host_vec = true; return true;
    case KB_F_EX: case KB_F_EY: case KB_F_EZ: case KB_F_HX: case KB_F_HY: case KB_F_HZ: {
      if (h->kind != KB_FDTD3D) return false;
      const int64_t M = h->N + 1;
      *dev = h->F[h->cur][field - KB_F_EX]; *bytes = M * M * M * 4;
      *rows = M * M;
      *pitch = h->pitch;
      return true;
    }
    case KB_F_PROBE:
      if (h->kind != KB_FDTD3D) return false;
      *dev = h->probe; *bytes = (size_t)h->pcap * 4; return true;
    case KB_F_STEP:
      if (h->kind != KB_FDTD3D) return false;
      *dev = reinterpret_cast<float *>(h->step); *bytes = 8; return true;
    case KB_F_W: case KB_F_SGSTATS: case KB_F_RESID:
    case KB_F_SG_X: case KB_F_SG_A1: case KB_F_SG_A2: case KB_F_SG_A3: case KB_F_SG_Z1: case KB_F_SG_Z2:
    case KB_F_SG_Z3: case KB_F_SG_Y: case KB_F_SG_TGT: case KB_F_SG_G4: case KB_F_SG_G1: case KB_F_SG_G2:
    case KB_F_SG_G3: case KB_F_SG_GRAD:
      if (h->kind != KB_HEAT2D_SURROGATE) return false;
      return sg_field(h, field, dev, bytes);
    case KB_F_REDLOG:
      if (!h->redlog) return false;
      *dev = reinterpret_cast<float *>(h->redlog); *bytes = (size_t)kRedLogCap * 4 * sizeof(double); return true;
    case KB_F_REDCOUNT:
      if (!h->redcount) return false;
      *dev = reinterpret_cast<float *>(h->redcount); *bytes = sizeof(long long); return true;
  }
  return false;
}

int check_heat_coeffs(const double *c, int nc, int layers3d, HeatCoef *k) {
  double cc = 1e-3, Rx = 1, Ry = 1, Rz = 10, Tamb = 300;
  if (nc != 0 && nc != 5) return fail(KB_EINVAL, "heat coefficients: expected 5 (c, Rx, Ry, Rz, Tamb), got %d", nc);
  if (nc == 5) { cc = c[0]; Rx = c[1]; Ry = c[2]; Rz = c[3]; Tamb = c[4]; }
  if (!(cc > 0) || !(Rx > 0) || !(Ry > 0) || !(Rz > 0) || !std::isfinite(Tamb))
    return fail(KB_EINVAL, "heat coefficients must be positive and finite");
  const double diag = cc * (2 / Rx + 2 / Ry + (layers3d ? 3 : 1) / Rz);
  if (!(diag < 1)) return fail(KB_EINVAL, "unstable heat step: c*(2/Rx+2/Ry+%s/Rz) = %g >= 1", layers3d ? "3" : "1", diag);
  k->cP = (float)cc;
  k->cx = (float)(cc / Rx);
  k->cy = (float)(cc / Ry);
  k->cz = (float)(cc / Rz);
  k->Tamb = (float)Tamb;
  return KB_OK;
}

}  // namespace

extern "C" {

int kb_abi_version(void) { return 2; }

int kb_stream_probe(int nin, int nout, int64_t n, void *workspace, size_t ws_bytes, void *stream, int reps,
                    double *seconds) {
  g_err.clear();
  if (!seconds || !workspace) return fail(KB_EINVAL, "null argument");
  if (nin < 1 || nin > 8 || nout < 1 || nout > 8) return fail(KB_EINVAL, "1 <= nin, nout <= 8");
  if (n < 4 || n % 4 != 0) return fail(KB_EINVAL, "n must be a positive multiple of 4");
  if (reps < 1) return fail(KB_EINVAL, "reps must be >= 1");
  if (ws_bytes < (size_t)(nin + nout) * (size_t)n * 4) return fail(KB_ENOMEM, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(KB_EINVAL, "workspace must be 256-byte aligned");
  const hipError_t e = stream_probe(nin, nout, n, static_cast<float *>(workspace),
                                    reinterpret_cast<hipStream_t>(stream), reps, seconds);
  if (e != hipSuccess) return fail(KB_EHIP, "stream probe: %s", hipGetErrorString(e));
  return KB_OK;
}

const char *kb_last_error(void) { return g_err.c_str(); }

size_t kb_workspace_bytes(int problem, const int64_t *shape, int ndim) {
  Layout L;
  size_t off[29] = {0};
  if (!layout(problem, shape, ndim, L, off)) return 0;
  return L.total;
}

int kb_kernels_per_iter(const kb_problem *h) { return h ? h->K : fail(KB_EINVAL, "null handle"); }

int kb_create(int problem, const int64_t *shape, int ndim, const double *coeffs, int ncoeffs, uint64_t seed,
              void *workspace, size_t ws_bytes, void *stream, kb_problem **out) {
  g_err.clear();
  if (!out) return fail(KB_EINVAL, "out is NULL");
  *out = nullptr;
  if (ncoeffs < 0 || (ncoeffs > 0 && !coeffs)) return fail(KB_EINVAL, "bad coefficient array");
  Layout Lay;
  size_t off[29] = {0};
  if (!layout(problem, shape, ndim, Lay, off)) return fail(KB_EINVAL, "invalid problem %d or shape", problem);
  if (!workspace || ws_bytes < Lay.total)
    return fail(KB_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, Lay.total);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(KB_ENOMEM, "workspace must be %zu-byte aligned", kAlign);

  kb_problem *h = new (std::nothrow) kb_problem();
  if (!h) return fail(KB_ENOMEM, "host allocation failed");
  h->kind = problem;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->ws = static_cast<unsigned char *>(workspace);
  h->ws_bytes = ws_bytes;
  auto P = [&](size_t o) { return reinterpret_cast<float *>(h->ws + o); };
  h->partials = reinterpret_cast<double *>(h->ws + off[3]);
  h->red = reinterpret_cast<double *>(h->ws + off[4]);
  if (problem != KB_HEAT2D_SURROGATE) {
    h->redlog = reinterpret_cast<double *>(h->ws + off[16]);
    h->redcount = reinterpret_cast<long long *>(h->ws + off[17]);
  }

  int rc = KB_OK;
  auto bail = [&](int code) { kb_destroy(h); return code; };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(KB_EHIP, "hipGetDevice failed"));
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return bail(fail(KB_EHIP, "hipEventCreate failed"));
  if (hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(KB_EHIP, "hipStreamCreateWithFlags failed"));

  switch (problem) {
    case KB_HEAT2D:
    case KB_HEAT3D: {
      const bool d3 = problem == KB_HEAT3D;
      if ((rc = check_heat_coeffs(coeffs, ncoeffs, d3, &h->hk)) != KB_OK) return bail(rc);
      h->nz = d3 ? shape[0] : 1;
      h->ny = shape[d3 ? 1 : 0];
      h->nx = shape[d3 ? 2 : 1];
      h->Tbuf[0] = P(off[0]); h->Tbuf[1] = P(off[1]); h->P = P(off[2]);
      h->K = 1;
      if ((rc = enqueue_init(h, h->Tbuf[0], h->nz * h->ny * h->nx, seed, kTagT0, 0, 323.0, 343.0)) ||
          (rc = enqueue_init(h, h->P, h->ny * h->nx, seed, kTagP, 0, 0.0, 1.0)))
        return bail(rc);
      break;
    }
    case KB_HEAT2D_SURROGATE: {
      if (ncoeffs != 0 && ncoeffs != 5 && ncoeffs != 8)
        return bail(fail(KB_EINVAL, "surrogate coeffs: {c, Rx, Ry, Rz, Tamb[, s, threshold, k]}"));
      if ((rc = check_heat_coeffs(coeffs, ncoeffs == 8 ? 5 : ncoeffs, 0, &h->hk)) != KB_OK) return bail(rc);
      std::string err;
      if ((rc = sg_create(h, shape, ndim, coeffs, ncoeffs, seed, err)) != KB_OK)
        return bail(fail(rc, "%s", err.c_str()));
      if ((rc = enqueue_init(h, h->Tbuf[0], h->ny * h->nx, seed, kTagT0, 0, 323.0, 343.0)))
        return bail(rc);
      {
        // the surrogate workload's power: uniform plus Gaussian hot spots
        Launch L;
        make_hot_spots(L, host_hot_spots(h->P, (int)h->ny, (int)h->nx, seed));
        if (hipLaunchKernel(L.func, L.grid, L.block, L.params(), 0, h->stream) != hipSuccess)
          return bail(fail(KB_EHIP, "hot-spot initialisation failed"));
      }
      if (sg_power_changed(h) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
        return bail(fail(KB_EHIP, "surrogate set-up failed"));
      break;
    }
    case KB_HEAT2D_MULTI: {
      if ((rc = check_heat_coeffs(coeffs, ncoeffs, 0, &h->hk)) != KB_OK) return bail(rc);
      h->G = (int)shape[0];
      h->grid_shape.assign(shape, shape + ndim);
      h->Tbuf[0] = P(off[0]); h->Tbuf[1] = P(off[1]); h->P = P(off[2]);
      h->grids_d = reinterpret_cast<GridDesc *>(h->ws + off[14]);
      h->block_start_d = reinterpret_cast<int *>(h->ws + off[15]);
      std::vector<GridDesc> gd(h->G);
      std::vector<int> bs(h->G + 1);
      long long offc = 0;
      int blocks = 0;
      for (int g = 0; g < h->G; ++g) {
        const int ny = (int)shape[1 + 2 * g], nx = (int)shape[2 + 2 * g];
        const int tx = (nx + kMultiBX - 1) / kMultiBX, ty = (ny + kMultiBY - 1) / kMultiBY;
        gd[g] = GridDesc{offc, ny, nx, tx, blocks};
        bs[g] = blocks;
        blocks += tx * ty;
        offc += (long long)ny * nx;
      }
      bs[h->G] = blocks;
      h->total_blocks = blocks;
      h->total_cells = offc;
      h->K = 1;
      // strip tiling: 64 columns x kStripTileY rows per block
      h->grids2_d = reinterpret_cast<GridDesc *>(h->ws + off[18]);
      h->block_grid_d = reinterpret_cast<int *>(h->ws + off[19]);
      std::vector<GridDesc> gd2(h->G);
      std::vector<int> bg;
      for (int g = 0; g < h->G; ++g) {
        const int tx = (gd[g].nx + 63) / 64, ty = (gd[g].ny + kStripTileY - 1) / kStripTileY;
        gd2[g] = GridDesc{gd[g].off, gd[g].ny, gd[g].nx, tx, (int)bg.size()};
        bg.insert(bg.end(), (size_t)tx * ty, g);
      }
      h->total_blocks2 = (int)bg.size();
      // temporal-blocking tilings: (64 - 2t) x (64 or 128 - 2t) output
      // tiles, t = 1..8; block0 counts from the start of each tiling's table
      h->grid_bar_d = reinterpret_cast<unsigned *>(h->ws + off[22]);
      h->grids_tb_d = reinterpret_cast<GridDesc *>(h->ws + off[20]);
      h->block_grid_tb_d = reinterpret_cast<int *>(h->ws + off[21]);
      std::vector<GridDesc> gdt((size_t)kMtTilings * h->G);
      std::vector<int> bgt;
      for (int sh = 0; sh < kMtShapes; ++sh)
        for (int t = 1; t <= kMtMaxDepth; ++t) {
          const int q = multi_tb_index(sh, t), tile_x = multi_tb_tile_x(sh, t), tile_y = multi_tb_tile_y(sh, t);
          h->tb_start[q] = (int)bgt.size();
          for (int g = 0; g < h->G; ++g) {
            const int tx = (gd[g].nx + tile_x - 1) / tile_x, ty = (gd[g].ny + tile_y - 1) / tile_y;
            gdt[(size_t)q * h->G + g] = GridDesc{gd[g].off, gd[g].ny, gd[g].nx, tx, (int)bgt.size() - h->tb_start[q]};
            bgt.insert(bgt.end(), (size_t)tx * ty, g);
          }
        }
      h->tb_start[kMtTilings] = (int)bgt.size();
      if (hipMemcpy(h->grids_d, gd.data(), gd.size() * sizeof(GridDesc), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(h->block_start_d, bs.data(), bs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(h->grids2_d, gd2.data(), gd2.size() * sizeof(GridDesc), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(h->block_grid_d, bg.data(), bg.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(h->grids_tb_d, gdt.data(), gdt.size() * sizeof(GridDesc), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(h->block_grid_tb_d, bgt.data(), bgt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(KB_EHIP, "grid table upload failed"));
      if ((rc = enqueue_init(h, h->Tbuf[0], offc, seed, kTagT0, 0, 323.0, 343.0)) ||
          (rc = enqueue_init(h, h->P, offc, seed, kTagP, 0, 0.0, 1.0)))
        return bail(rc);
      break;
    }
    case KB_SKELETON: {
      if (ncoeffs < 1) return bail(fail(KB_EINVAL, "skeleton needs coeffs {K[, a_1..a_K, b_1..b_K]}"));
      const int K = (int)coeffs[0];
      if ((double)K != coeffs[0] || K < 1 || K > kMaxK) return bail(fail(KB_EINVAL, "skeleton K must be 1..%d", kMaxK));
      if (ncoeffs != 1 && ncoeffs != 1 + 2 * K) return bail(fail(KB_EINVAL, "skeleton coeffs: 1 or 1+2K values"));
      h->K = K;
      h->n = shape[0];
      h->x = P(off[0]);
      h->a.resize(K);
      h->b.resize(K);
      for (int k = 0; k < K; ++k) {
        h->a[k] = ncoeffs > 1 ? (float)coeffs[1 + k] : host_uniform(seed, kTagA, k, 0.9, 1.0);
        h->b[k] = ncoeffs > 1 ? (float)coeffs[1 + K + k] : host_uniform(seed, kTagB, k, -0.01, 0.01);
      }
      if ((rc = enqueue_init(h, h->x, h->n, seed, kTagX0, 0, -1.0, 1.0))) return bail(rc);
      break;
    }
    case KB_FDTD3D: {
      if (ncoeffs != 3 && ncoeffs != 6)
        return bail(fail(KB_EINVAL, "fdtd coeffs: {courant, width, delay[, i, j, k]}"));
      const int N = (int)shape[0];
      const double courant = coeffs[0], width = coeffs[1], delay = coeffs[2];
      if (!(courant > 0) || !(courant < 1.0 / std::sqrt(3.0)))
        return bail(fail(KB_EINVAL, "courant number %g outside (0, 1/sqrt(3))", courant));
      h->N = N;
      h->pitch = (int)fdtd_pitch(N);
      h->dt = (float)courant;
      h->K = 2;                                 // the fused step and the source
      for (int f = 0; f < 6; ++f) {
        h->F[0][f] = P(off[5 + f]);
        h->F[1][f] = P(off[23 + f]);
      }
      h->g = P(off[11]);
      h->probe = P(off[12]);
      h->pcap = (int)(ndim == 2 ? shape[1] : kDefaultProbe);
      h->step = reinterpret_cast<long long *>(h->ws + off[13]);
      h->done = reinterpret_cast<unsigned *>(h->ws + off[13] + 8);
      int si, sj, sk;
      if (ncoeffs == 6) {
        si = (int)coeffs[3]; sj = (int)coeffs[4]; sk = (int)coeffs[5];
        if (si < 1 || si > N - 1 || sj < 1 || sj > N - 1 || sk < 0 || sk > N - 1)
          return bail(fail(KB_EINVAL, "source node (%d,%d,%d) is not an interior Ez node", si, sj, sk));
      } else {
        si = 2 + (int)host_randint(seed, kTagSrc, 0, N - 3);
        sj = 2 + (int)host_randint(seed, kTagSrc, 1, N - 3);
        sk = 1 + (int)host_randint(seed, kTagSrc, 2, N - 2);
      }
      h->src_ijk[0] = si; h->src_ijk[1] = sj; h->src_ijk[2] = sk;
      const long long M = N + 1;
      h->src = ((long long)sk * M + sj) * h->pitch + si;
      // amplitude table: g(n) = exp(-((n - delay)/width)^2) rounded to float,
      // up to the first step after which every value rounds to zero.
      std::vector<float> gt;
      if (width > 0) {
        const double last = delay + width * std::sqrt(104.0);
        if (!(last < kGCap - 1)) return bail(fail(KB_EINVAL, "source pulse longer than %d steps", kGCap));
        const int len = (int)std::ceil(last) + 1;
        gt.resize(len);
        for (int n = 0; n < len; ++n) {
          const double x = ((double)n - delay) / width;
          gt[n] = (float)std::exp(-(x * x));
        }
      }
      h->glen = (int)gt.size();
      for (int q = 0; q < 2; ++q)
        for (int f = 0; f < 6; ++f)
          if (hipMemsetAsync(h->F[q][f], 0, M * M * h->pitch * 4, h->stream) != hipSuccess)
            return bail(fail(KB_EHIP, "hipMemsetAsync failed"));
      if (hipMemsetAsync(h->probe, 0, (size_t)(h->pcap > 0 ? h->pcap : 1) * 4, h->stream) != hipSuccess ||
          hipMemsetAsync(h->step, 0, 16, h->stream) != hipSuccess)
        return bail(fail(KB_EHIP, "hipMemsetAsync failed"));
      if (h->glen > 0 && hipMemcpyAsync(h->g, gt.data(), gt.size() * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return bail(fail(KB_EHIP, "source table upload failed"));
      if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(KB_EHIP, "hipStreamSynchronize failed"));
      break;
    }
  }
  if (h->redcount && hipMemsetAsync(h->redcount, 0, sizeof(long long), h->stream) != hipSuccess)
    return bail(fail(KB_EHIP, "hipMemsetAsync failed"));
  *out = h;
  return KB_OK;
}

int kb_set_option(kb_problem *h, int option, int64_t value) {
  if (!h) return fail(KB_EINVAL, "null handle");
  switch (option) {
    case KB_OPT_BUILDER:
      if (value != 0 && value != 1) return fail(KB_EINVAL, "builder must be 0 or 1");
      if (h->builder != value) clear_cache(h);   // cached graphs belong to the other builder
      h->builder = (int)value;
      break;
    case KB_OPT_TILE: {
      bool ok = false;
      if (h->kind == KB_HEAT2D)
        ok = (value >= 0 && value <= 7) || (value >= 8 && value <= 14 && h->nx % 4 == 0) || (value >= 15 && value <= 23);
      else if (h->kind == KB_HEAT3D)
        ok = value == 0 || value == 1 || (((value >= 2 && value <= 4) || (value >= 6 && value <= 10)) && h->nx % 4 == 0) ||
             ((value == 5 || value == 11) && h->nz <= 8);
      else if (h->kind == KB_SKELETON) ok = value >= 0 && value <= 3;
      else if (h->kind == KB_FDTD3D) ok = value >= 0 && value <= 10;
      else if (h->kind == KB_HEAT2D_SURROGATE) ok = value >= 0 && value <= 2;
      else if (h->kind == KB_HEAT2D_MULTI) ok = value >= 0 && value <= 6;
      else ok = value == 0;
      if (!ok) return fail(KB_EINVAL, "kernel variant %lld not available for this problem", (long long)value);
      if (h->tile != value) clear_cache(h);
      h->tile = (int)value;
      if (h->kind == KB_HEAT2D_SURROGATE) h->K = sg_kernels_per_block(h);
      if (h->kind == KB_FDTD3D) h->K = fdtd_kernels_per_iter(h);
      break;
    }
    case KB_OPT_TDEPTH: {
      if (h->kind != KB_HEAT2D && h->kind != KB_HEAT3D && h->kind != KB_HEAT2D_MULTI && h->kind != KB_FDTD3D &&
          value != 1)
        return fail(KB_EINVAL, "temporal depth > 1 only for KB_HEAT2D, KB_HEAT3D, KB_HEAT2D_MULTI and KB_FDTD3D");
      // FDTD: two steps per launch with variants 8-10, three with 9 and 10
      // (whole rows, N <= 256); the other variants advance one step per
      // launch whatever the depth
      const int maxd = h->kind == KB_HEAT3D ? heat3d_tb_max_depth()
                     : h->kind == KB_HEAT2D_MULTI ? kMtMaxDepth
                     : h->kind == KB_FDTD3D ? 3 : heat2d_tile_max_depth();
      if (value < 1 || value > maxd) return fail(KB_EINVAL, "temporal depth must be 1..%d", maxd);
      if (h->tdepth != value) clear_cache(h);
      h->tdepth = (int)value;
      if (h->kind == KB_FDTD3D) h->K = fdtd_kernels_per_iter(h);
      break;
    }
    case KB_OPT_GRAPH_CACHE:
      if (value != 0 && value != 1) return fail(KB_EINVAL, "graph cache must be 0 or 1");
      h->cache = (int)value;
      if (!value) clear_cache(h);
      break;
    case KB_OPT_MAX_NODES:
      if (value < 1) return fail(KB_EINVAL, "max nodes must be >= 1");
      h->max_nodes = value;
      break;
    case KB_OPT_GRAPH_UPDATE:
      if (value != 0 && value != 1) return fail(KB_EINVAL, "graph update must be 0 or 1");
      h->graph_update = (int)value;
      break;
    case KB_OPT_PERSISTENT: {
      if (value != 0 && value != 1) return fail(KB_EINVAL, "persistent must be 0 or 1");
      if (value && h->kind != KB_HEAT2D_MULTI) return fail(KB_EINVAL, "persistent runs only for KB_HEAT2D_MULTI");
      if (value) {
        int coop = 0;
        HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device));
        if (!coop) return fail(KB_EHIP, "device has no cooperative launch");
      }
      h->persistent = (int)value;
      break;
    }
    case KB_OPT_SPIN_LIMIT:
      if (value < 0 || value > INT32_MAX) return fail(KB_EINVAL, "spin limit must be 0..2^31-1");
      h->spin_limit = value;
      break;
    case KB_OPT_REDUCE_EVERY:
      if (h->kind == KB_HEAT2D_SURROGATE) return fail(KB_EINVAL, "the surrogate has its own residual check");
      if (value < 0) return fail(KB_EINVAL, "reduction interval must be >= 0");
      clear_cache(h);
      h->red_every = value;
      h->step_count = 0;
      HIPCHK(hipMemsetAsync(h->redcount, 0, sizeof(long long), h->stream));
      break;
    default:
      return fail(KB_EINVAL, "unknown option %d", option);
  }
  return KB_OK;
}

// One cooperative launch of the persistent many-grid kernel for n steps.
int run_persistent(kb_problem *h, int64_t n_steps) {
  if (h->red_every > 0) return fail(KB_EINVAL, "in-chain reductions are not available in a persistent run");
  const int t = h->tdepth;
  const int64_t nfull = n_steps / t;
  const int rem = (int)(n_steps % t);
  if (nfull > (int64_t)1 << 30) return fail(KB_EINVAL, "too many steps for one persistent launch");
  const void *f = multi_persistent_fn();
  if (h->persist_blocks == 0) {
    int per_cu = 0, cus = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    // Resident blocks, a multiple of the XCD count (the kernel splits the
    // tile list into one part per XCD).  At most half of what the occupancy
    // query reports: the query counts registers and LDS but not the scalar
    // register file, which limits this kernel (about 106 SGPRs) to 7 waves
    // per SIMD, not the 8 the query assumes; a grid that is not entirely
    // resident would never pass its first barrier.  And at most 2 per CU:
    // every block adds a writeback and an invalidate to each barrier
    // (measured at depth 1: 45 us per step with 2 per CU, 54 with 4, 50
    // with 1; equal at depth 6 for 2 and 4).
    h->persist_blocks = std::min(2, std::max(1, per_cu / 2)) * cus / kXcds * kXcds;
    if (h->persist_blocks < kXcds) return fail(KB_EHIP, "persistent kernel does not fit the device");
  }
  int most = 0;                                 // tiles of the busiest super-step
  for (int d : {t, rem})
    if (d > 0) most = std::max(most, h->tb_start[d] - h->tb_start[d - 1]);
  const int blocks = std::max(kXcds, std::min(h->persist_blocks, (most + kXcds - 1) / kXcds * kXcds));
  MultiPersistArgs a{};
  a.T0 = h->Tbuf[h->cur];
  a.T1 = h->Tbuf[1 - h->cur];
  a.P = h->P;
  a.grids = h->grids_tb_d;                      // region shape 0 (64 x 64): tilings 0 .. kMtMaxDepth-1
  a.block_grid = h->block_grid_tb_d;
  for (int d = 0; d <= kMtMaxDepth; ++d) a.tb_start[d] = h->tb_start[d];
  a.G = h->G;
  a.tdepth = t;
  a.nfull = (int)nfull;
  a.rem = rem;
  a.bar = h->grid_bar_d;
  // polls of a barrier wait before it gives up: about a second (one poll is
  // an uncached load and a short sleep), more for huge super-steps
  a.spin_limit = h->spin_limit > 0 ? (unsigned)h->spin_limit
               : (unsigned)std::min<int64_t>(INT32_MAX, std::max<int64_t>(1 << 20, h->total_cells * t >> 14));
  a.k = h->hk;
  void *args[] = {&a};
  kb_timing tm{};
  HIPCHK(hipMemsetAsync(h->grid_bar_d, 0, kBarWords * sizeof(unsigned), h->stream));
  HIPCHK(hipEventRecord(h->ev0, h->stream));
  if (n_steps > 0) HIPCHK(hipLaunchCooperativeKernel(f, dim3(blocks), dim3(256), args, 0, h->stream));
  HIPCHK(hipEventRecord(h->ev1, h->stream));
  unsigned err = 0;
  HIPCHK(hipMemcpyAsync(&err, h->grid_bar_d + 2, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int64_t nsuper = nfull + (rem > 0 ? 1 : 0);
  if (nsuper & 1) h->cur ^= 1;
  h->step_count += n_steps;
  h->host_steps += n_steps;
  tm.n_kernel_launches = n_steps > 0 ? 1 : 0;
  h->last = tm;
  h->timed = true;
  if (err) return fail(KB_EHIP, "persistent kernel: a grid barrier wait timed out; the state is invalid");
  return KB_OK;
}

int kb_run(kb_problem *h, int64_t n_steps, int64_t batch_b) {
  if (!h) return fail(KB_EINVAL, "null handle");
  if (n_steps < 0 || batch_b < 0) return fail(KB_EINVAL, "n_steps and batch_b must be >= 0");
  if (h->persistent) return run_persistent(h, n_steps);
  const int depth = iter_depth(h);
  const int64_t n_iter = n_steps / depth;
  const int64_t rem_steps = n_steps % depth;
  kb_timing t{};
  int status = KB_OK;
  const bool pp = alternates(h);

  if (batch_b > 0 && (batch_b > h->max_nodes / h->K))
    return fail(KB_EINVAL, "batch of %lld iterations x %d kernels exceeds %lld graph nodes", (long long)batch_b, h->K,
                (long long)h->max_nodes);

  // in-chain reductions: every reduction point (a multiple of m steps since
  // the option was set) must fall on an iteration boundary
  if (h->red_every > 0 && (rem_steps != 0 || h->red_every % depth != 0 || h->step_count % depth != 0))
    return fail(KB_EINVAL, "in-chain reductions need m and the steps run so far to be multiples of the "
                           "temporal depth %d, and n_steps too", depth);

  // Replay j starts from buffer parity cur_j and phase ph_j = steps since
  // the last reduction point; both are periodic in j, and each distinct
  // (parity, phase) pair has its own executable graph.
  using Key = std::tuple<int64_t, int, int, int, int64_t>;
  int64_t nb = 0, peel = n_iter;
  std::map<std::pair<int, int64_t>, hipGraphExec_t> execs;
  if (batch_b > 0 && n_iter >= batch_b) {
    nb = n_iter / batch_b;
    peel = n_iter % batch_b;
    const int64_t m = h->red_every;
    const bool flip = pp && (batch_b & 1);
    std::vector<std::pair<int, int64_t>> need;
    int c = h->cur;
    int64_t ph = m > 0 ? h->step_count % m : 0;
    const int64_t period = 2 * (m > 0 ? m : 1);
    for (int64_t j = 0; j < std::min(nb, period); ++j) {
      // the buffer set a replay starts from: it alternates between replays
      // only if the state moves every iteration and b is odd (FDTD's
      // in-place kernels run on whichever set is current)
      std::pair<int, int64_t> q{c, ph};
      if (std::find(need.begin(), need.end(), q) == need.end()) need.push_back(q);
      if (flip) c ^= 1;
      if (m > 0) ph = (ph + batch_b * depth) % m;
    }
    if (need.size() > 64)
      return fail(KB_EINVAL, "batch %lld and reduction interval %lld need %zu distinct graphs (max 64)",
                  (long long)batch_b, (long long)m, need.size());
    size_t free0 = 0, free1 = 0, total = 0;
    const bool have_mem = hipMemGetInfo(&free0, &total) == hipSuccess;
    const double t0 = now_s();
    for (const auto &q : need) {
      const Key key = std::make_tuple(batch_b, depth, h->tile, q.first, q.second);
      auto it = h->cache_map.find(key);
      if (it != h->cache_map.end()) { execs[q] = it->second; continue; }
      hipGraphExec_t ex = nullptr;
      int rc = build_graph(h, batch_b, depth, q.first, q.second, &ex);
      if (rc != KB_OK) { status = KB_WFALLBACK; break; }
      h->cache_map[key] = ex;
      execs[q] = ex;
      t.n_graphs_built++;
    }
    if (t.n_graphs_built > 0) {
      hipError_t e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) return fail(KB_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    t.t_create_s = now_s() - t0;
    if (have_mem && t.n_graphs_built > 0 && hipMemGetInfo(&free1, &total) == hipSuccess)
      t.graph_mem_bytes = (int64_t)free0 - (int64_t)free1;
    if (status == KB_WFALLBACK) { nb = 0; peel = n_iter; }
  }

  HIPCHK(hipEventRecord(h->ev0, h->stream));
  for (int64_t j = 0; j < nb; ++j) {
    const int64_t ph = h->red_every > 0 ? h->step_count % h->red_every : 0;
    hipGraphExec_t ex = execs[std::make_pair(h->cur, ph)];
    HIPCHK(hipGraphLaunch(ex, h->stream));
    if (pp && (batch_b & 1)) h->cur ^= 1;
    h->step_count += batch_b * depth;
  }
  for (int64_t j = 0; j < peel; ++j) {
    int rc = launch_iter(h, depth, h->stream);
    if (rc != KB_OK) return rc;
  }
  for (int64_t j = 0; j < rem_steps; ++j) {
    int rc = launch_iter(h, 1, h->stream);
    if (rc != KB_OK) return rc;
  }
  HIPCHK(hipEventRecord(h->ev1, h->stream));
  t.n_graph_launches = nb;
  t.n_nodes = nb > 0 ? batch_b * h->K : 0;
  t.n_peeled = peel + rem_steps;
  t.n_kernel_launches = (peel + rem_steps) * h->K;
  h->last = t;
  h->timed = true;
  h->host_steps += n_steps;
  if (!h->cache && !h->cache_map.empty()) {
    HIPCHK(hipStreamSynchronize(h->stream));
    clear_cache(h);
  }
  return status;
}

int kb_last_timing(kb_problem *h, kb_timing *out) {
  if (!h || !out) return fail(KB_EINVAL, "null argument");
  if (!h->timed) return fail(KB_ESTATE, "no kb_run yet");
  HIPCHK(hipEventSynchronize(h->ev1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  *out = h->last;
  out->t_exec_s = ms * 1e-3;
  out->t_update_s = h->t_update_s;
  out->n_graphs_updated = h->n_updated;
  return KB_OK;
}

int kb_read(kb_problem *h, int field, void *dst, size_t bytes, int dst_on_device) {
  if (!h || !dst) return fail(KB_EINVAL, "null argument");
  float *dev = nullptr;
  size_t need = 0, rows = 0, pitch = 0;
  bool hv = false;
  if (!field_info(h, field, &dev, &need, &hv, &rows, &pitch))
    return fail(KB_EINVAL, "field %d not available", field);
  if (bytes != need) return fail(KB_EINVAL, "field %d has %zu bytes, got %zu", field, need, bytes);
  HIPCHK(hipStreamSynchronize(h->stream));
  if (hv) {
    const std::vector<float> &v = field == KB_F_A ? h->a : h->b;
    if (dst_on_device) HIPCHK(hipMemcpy(dst, v.data(), bytes, hipMemcpyHostToDevice));
    else std::memcpy(dst, v.data(), bytes);
    return KB_OK;
  }
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (rows) {
    const size_t w = bytes / rows;   // dense row bytes
    HIPCHK(hipMemcpy2D(dst, w, dev, pitch * sizeof(float), w, rows, kind));
  } else {
    HIPCHK(hipMemcpy(dst, dev, bytes, kind));
  }
  return KB_OK;
}

int kb_write(kb_problem *h, int field, const void *src, size_t bytes, int src_on_device) {
  if (!h || !src) return fail(KB_EINVAL, "null argument");
  if (field >= KB_F_SG_X && field <= KB_F_SG_GRAD) return fail(KB_EINVAL, "field %d is read only", field);
  float *dev = nullptr;
  size_t need = 0, rows = 0, pitch = 0;
  bool hv = false;
  if (!field_info(h, field, &dev, &need, &hv, &rows, &pitch))
    return fail(KB_EINVAL, "field %d not available", field);
  if (bytes != need) return fail(KB_EINVAL, "field %d has %zu bytes, got %zu", field, need, bytes);
  HIPCHK(hipStreamSynchronize(h->stream));
  if (hv) {
    std::vector<float> &v = field == KB_F_A ? h->a : h->b;
    if (src_on_device) HIPCHK(hipMemcpy(v.data(), src, bytes, hipMemcpyDeviceToHost));
    else std::memcpy(v.data(), src, bytes);
    // a_k, b_k are baked into graph nodes
    const double t0 = now_s();
    if (h->graph_update) h->n_updated = update_cached(h);
    else clear_cache(h);
    h->t_update_s = now_s() - t0;
    return KB_OK;
  }
  const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (rows) {
    const size_t w = bytes / rows;   // dense row bytes; the padding columns stay zero
    HIPCHK(hipMemcpy2D(dev, pitch * sizeof(float), src, w, w, rows, kind));
  } else {
    HIPCHK(hipMemcpy(dev, src, bytes, kind));
  }
  if (h->kind == KB_FDTD3D && field >= KB_F_EX && field <= KB_F_HZ) {
    // the cavity's i = N column is kept equal in both field sets (no step
    // changes E, Hy or Hz there, and every kernel that writes a whole set
    // copies them): mirror the written column into the other set
    float *other = h->F[1 - h->cur][field - KB_F_EX];
    HIPCHK(hipMemcpy2D(other + h->N, pitch * sizeof(float), dev + h->N, pitch * sizeof(float), sizeof(float), rows,
                       hipMemcpyDeviceToDevice));
  }
  if (h->kind == KB_HEAT2D_SURROGATE && (field == KB_F_W || field == KB_F_P)) {
    // derived device data: the packed bf16 weights, the power sum
    HIPCHK(field == KB_F_W ? sg_repack(h) : sg_power_changed(h));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return KB_OK;
}

int kb_reduce(kb_problem *h, double *out, int nout) {
  if (!h || !out) return fail(KB_EINVAL, "null argument");
  hipError_t e = hipSuccess;
  int nres = 1;
  if (pingpong(h)) {
    const long long n = h->kind == KB_HEAT2D_MULTI ? h->total_cells : h->nz * h->ny * h->nx;
    e = reduce_sum(h->Tbuf[h->cur], n, h->partials, h->red, h->stream);
  } else if (h->kind == KB_SKELETON) {
    e = reduce_sum(h->x, h->n, h->partials, h->red, h->stream);
  } else {
    // padded arrays: the padding columns hold zeros and add nothing
    const long long n = (long long)(h->N + 1) * (h->N + 1) * h->pitch;
    float *const *F = h->F[h->cur];
    const float *E[3] = {F[0], F[1], F[2]};
    const float *H[3] = {F[3], F[4], F[5]};
    e = reduce_sumsq(E, 3, n, h->partials, h->red, h->stream);
    if (e == hipSuccess) e = reduce_sumsq(H, 3, n, h->partials, h->red + 1, h->stream);
    nres = 2;
  }
  if (e != hipSuccess) return fail(KB_EHIP, "reduction launch: %s", hipGetErrorString(e));
  if (nout < nres) return fail(KB_EINVAL, "need room for %d results", nres);
  double tmp[2];
  HIPCHK(hipMemcpyAsync(tmp, h->red, nres * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int q = 0; q < nres; ++q) out[q] = tmp[q];
  return KB_OK;
}

int kb_destroy(kb_problem *h) {
  if (!h) return KB_OK;
  int rc = KB_OK;
  if (hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(KB_EHIP, "hipStreamSynchronize failed in destroy");
  clear_cache(h);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->sg) sg_destroy(h);
  delete h;
  return rc;
}

}  // extern "C"
