// Internal declarations of libkbatch (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "kb.h"

namespace kb {

// ---------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea, Flood 2014), used for the seeded
// initial state.  Draw idx of stream (seed, tag) is output idx+1 of a
// SplitMix64 sequence whose state starts at seed ^ (tag << 48).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t splitmix(uint64_t seed, uint64_t tag, uint64_t idx) {
  uint64_t z = (seed ^ (tag << 48)) + (idx + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum Tag : uint64_t { kTagT0 = 1, kTagP = 2, kTagX0 = 3, kTagA = 4, kTagB = 5, kTagSrc = 6, kTagHot = 7 };

// Host-side uniform draw, rounded once to float (matches the device draw).
float host_uniform(uint64_t seed, uint64_t tag, uint64_t idx, double lo, double hi);
// Integer on [0, m) from the top 24 bits.
int64_t host_randint(uint64_t seed, uint64_t tag, uint64_t idx, int64_t m);

// ---------------------------------------------------------------------------
// One kernel launch: function, shape, and its single by-value argument
// struct.  The per-launch driver and both graph builders consume the same
// descriptors, so the two execution paths run identical kernels on
// identical arguments.
// ---------------------------------------------------------------------------
struct Launch {
  const void *func = nullptr;
  dim3 grid{1, 1, 1};
  dim3 block{1, 1, 1};
  unsigned lds = 0;
  alignas(16) unsigned char args[256];
  size_t args_size = 0;
  void *argv[1] = {nullptr};

  template <class A> void set(const void *f, dim3 g, dim3 b, unsigned shm, const A &a) {
    static_assert(sizeof(A) <= sizeof(args), "kernel argument struct too large");
    func = f; grid = g; block = b; lds = shm;
    std::memcpy(args, &a, sizeof(A));
    args_size = sizeof(A);
    argv[0] = args;
  }
  // argv points into this object; refresh after copies.
  void **params() { argv[0] = args; return argv; }
};

// ---------------------------------------------------------------------------
// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Kernels remap the hardware block id so that XCD x receives one contiguous
// run of logical blocks (a band of rows or planes), which keeps the halo
// rows/planes of neighbouring tiles in the same L2.  The grid is padded to a
// multiple of 8; logical ids past the end return.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kCUs = 256;                 // compute units of the MI355X (32 per XCD)

__device__ __forceinline__ int xcd_logical_block(int nblocks) {
  const int hw = blockIdx.x;
  const int per = (nblocks + kXcds - 1) / kXcds;
  return (hw % kXcds) * per + hw / kXcds;
}

inline int xcd_padded_grid(int nblocks) { return (nblocks + kXcds - 1) / kXcds * kXcds; }

// Value of the neighbouring lane of a full wave, by a DPP wave shift; the
// lane at the end of the wave reads 0 (callers clamp where that matters).
__device__ __forceinline__ float lane_west_open(float v) {   // lane - 1 (wave_shr:1)
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_east_open(float v) {   // lane + 1 (wave_shl:1)
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}


// ---------------------------------------------------------------------------
// Kernel argument structs (passed by value).
// ---------------------------------------------------------------------------
struct HeatCoef {
  float cP, cx, cy, cz, Tamb;   // c, c/Rx, c/Ry, c/Rz, Tamb rounded to float
};

struct Heat2DArgs {
  const float *T; float *out; const float *P;
  int ny, nx;
  HeatCoef k;
  int tdepth;                  // steps per launch (tile kernels)
  const int *flag;             // tile kernels: run only if *flag != 0 (null: always)
};

struct Heat3DArgs {
  const float *T; float *out; const float *P;   // P: plane of layer 0
  int nz, ny, nx;
  HeatCoef k;
  int tdepth = 1;                               // steps per launch (variant 5)
};
int heat3d_tb_max_depth();

struct GridDesc {               // one grid of the many-grid problem
  long long off;                // first cell in the concatenated arrays
  int ny, nx;
  int tiles_x;                  // tiles along x
  int block0;                   // first block of this grid
};

struct MultiArgs {
  const float *T; float *out; const float *P;
  const GridDesc *grids;
  const int *block_start;       // G+1 prefix sums of blocks per grid
  int G;
  HeatCoef k;
};

// Many-grid strip kernel: a block of 4 waves covers 64 columns x 32 rows of
// one grid; block -> grid by table.
constexpr int kStripRows = 8;                 // rows per wave
constexpr int kStripTileY = 4 * kStripRows;   // rows per block
struct MultiStripArgs {
  const float *T; float *out; const float *P;
  const GridDesc *grids;        // tiles_x / block0 of the 64 x 32 tiling
  const int *block_grid;        // grid of every block
  int nb;
  HeatCoef k;
};

// Many-grid temporal blocking: t <= kMtMaxDepth steps per launch over a
// region of at most multi_tb_region_x(s) columns x multi_tb_region_y(s)
// rows around an output tile of (region columns - 2t) x (region rows - 2t)
// cells; region shape s = 0 (64 x 64, 4 waves), 1 (64 x 128, 8 waves),
// 2 (128 x 64, two columns per lane, 4 waves) or 3 (128 x 128, two
// columns per lane, 8 waves); one block table per (s, t).
constexpr int kMtRegionX = 64, kMtMaxDepth = 8, kMtShapes = 4;
constexpr int kMtTilings = kMtShapes * kMtMaxDepth;
__host__ __device__ inline int multi_tb_region_x(int s) { return s >= 2 ? 128 : 64; }
__host__ __device__ inline int multi_tb_region_y(int s) { return (s & 1) ? 128 : 64; }
__host__ __device__ inline int multi_tb_tile_x(int s, int t) { return multi_tb_region_x(s) - 2 * t; }
__host__ __device__ inline int multi_tb_tile_y(int s, int t) { return multi_tb_region_y(s) - 2 * t; }
inline int multi_tb_index(int s, int t) { return s * kMtMaxDepth + t - 1; }
struct MultiTbArgs {
  const float *T; float *out; const float *P;
  const GridDesc *grids;        // tiles_x / block0 of the tiling at this depth
  const int *block_grid;        // grid of every block
  int nb, tdepth;
  HeatCoef k;
};
void make_multi_tb(Launch &L, const MultiTbArgs &a, int shape);

// Persistent many-grid run (one cooperative launch of 256-thread blocks):
// nfull super-steps of tdepth steps, then one of rem steps (if rem > 0),
// over the 64 x 64-region tilings.
struct MultiPersistArgs {
  float *T0, *T1;                  // T0 holds the state at entry
  const float *P;
  const GridDesc *grids;           // the G descriptors of each depth's tiling, depth 1 first
  const int *block_grid;           // block tables of those tilings, concatenated
  int tb_start[kMtMaxDepth + 1];   // entries of depth d: tb_start[d-1] .. tb_start[d]
  int G, tdepth, nfull, rem;
  unsigned *bar;                   // barrier words (kBarWords), zero at launch
  unsigned spin_limit;             // polls before a barrier wait gives up
  HeatCoef k;
};
const void *multi_persistent_fn();
// The persistent kernel's barrier words: [0] top arrival count, [1]
// generation, [2] error flag; the group counters at kBarStride * (1 + g),
// each on its own 128-byte line.
constexpr unsigned kBarGroups = 8, kBarStride = 32;
constexpr size_t kBarWords = (size_t)kBarStride * (1 + kBarGroups);

struct SkelArgs {
  float *x; long long n; float a, b;
};

struct FdtdArgs {
  float *Ex, *Ey, *Ez, *Hx, *Hy, *Hz;
  int N;        // cells per edge; nodes 0..N in each direction
  int P;        // row pitch in floats (multiple of 4, >= N+1)
  float dt;
};

// Fused H + E step: reads E^n, H^{n-1/2} from one buffer set and writes
// H^{n+1/2}, E^{n+1} to the other.
struct FdtdFusedArgs {
  const float *Ex, *Ey, *Ez, *Hx, *Hy, *Hz;
  float *oEx, *oEy, *oEz, *oHx, *oHy, *oHz;
  int N, P;
  float dt;
};
bool make_fdtd_fused(Launch &L, const FdtdFusedArgs &a, int kc, bool nt);   // kc: planes per thread (1, 8); nt: streaming stores (kc 1)

// Two steps per launch (temporal blocking): reads E^n, H^{n-1/2} from one
// buffer set and writes E^{n+2}, H^{n+3/2} to the other, applying the soft
// source (and recording the probe) after each of the two E updates; the
// device step counter is advanced by a separate launch.
struct FdtdTbArgs {
  const float *Ex, *Ey, *Ez, *Hx, *Hy, *Hz;
  float *oEx, *oEy, *oEz, *oHx, *oHy, *oHz;
  int N, P;
  float dt;
  int tk, ni, nj, nk;           // planes per block; tiles along i, j, k
  int si, sj, sk;               // source node (i, j, k)
  const float *g; int glen;     // amplitude per absolute step
  float *probe; int pcap;
  const long long *step;
  // whole-row kernels: the step counter they advance and the counter of
  // finished blocks (zero between launches) that says which block does it
  long long *step_w; unsigned *done;
  long long fs;                 // bytes from one field to the next within a set (three-step kernel)
};
bool make_fdtd_tb2(Launch &L, const FdtdTbArgs &a, bool nt);   // fills tk..nk itself
// Whole-row form (N <= 256, false otherwise): the iteration's one kernel
// (it also writes the i = N column at N = 256 and advances the step counter).
bool make_fdtd_tb2_rows(Launch &L, const FdtdTbArgs &a, bool nt, int form);   // form 0: 16 waves; 1: 12 waves, operands one plane ahead
bool make_fdtd_tb3_rows(Launch &L, const FdtdTbArgs &a, bool nt);             // three steps per launch, 12 waves
void make_fdtd_step_add(Launch &L, long long *step, int d);

struct SrcArgs {
  float *Ez; long long src;     // flat index of the source node
  const float *g; int glen;     // amplitude per absolute step
  float *probe; int pcap;
  long long *step;
};

struct InitArgs {
  float *out; long long n; unsigned long long seed, tag, offset;
  double lo, span;
};

// Power map with Gaussian hot spots: P ~ U[0,1) (stream kTagP) plus up to
// four spots whose parameters the host draws from stream kTagHot.
struct HotSpotArgs {
  float *out; int ny, nx; unsigned long long seed;
  int count;
  double cy[4], cx[4], amp[4], den[4];   // den = (2 sigma) sigma
};

// ---------------------------------------------------------------------------
// Kernel launchers / descriptor builders, defined in the .hip files.
// ---------------------------------------------------------------------------
void make_init(Launch &L, const InitArgs &a);
void make_hot_spots(Launch &L, const HotSpotArgs &a);
HotSpotArgs host_hot_spots(float *out, int ny, int nx, uint64_t seed);
void make_heat2d_direct(Launch &L, const Heat2DArgs &a);
bool make_heat2d_tile(Launch &L, const Heat2DArgs &a, int variant);   // false: bad variant
int heat2d_tile_max_depth();
bool make_heat2d_strip(Launch &L, const Heat2DArgs &a, int variant);
bool make_heat2d_region(Launch &L, const Heat2DArgs &a, int variant);  // 15-17; false: depth > 8
int heat2d_strip_max_depth();
bool make_heat3d(Launch &L, const Heat3DArgs &a, int variant);   // false: bad variant
bool make_heat2d_vec(Launch &L, const Heat2DArgs &a, int variant);  // false: bad variant / nx % 4
constexpr int kMultiBX = 64, kMultiBY = 4;   // tile of the many-grid kernel
void make_multi(Launch &L, const MultiArgs &a, int total_blocks);
void make_multi_strip(Launch &L, const MultiStripArgs &a);
void make_skeleton(Launch &L, const SkelArgs &a, int variant);
bool make_fdtd_h(Launch &L, const FdtdArgs &a, int variant);   // false: bad variant
bool make_fdtd_e(Launch &L, const FdtdArgs &a, int variant);
void make_fdtd_src(Launch &L, const SrcArgs &a);

// Surrogate problem (sg_api.hip).
struct SgState;
size_t sg_workspace_bytes(const int64_t *shape, int ndim);
int sg_create(kb_problem *h, const int64_t *shape, int ndim, const double *c, int nc, uint64_t seed,
              std::string &err);
void sg_destroy(kb_problem *h);
int sg_iter_depth(const kb_problem *h);
int sg_fill_iter(const kb_problem *h, int cur, Launch *L);
int sg_kernels_per_block(const kb_problem *h);
bool sg_field(const kb_problem *h, int field, float **dev, size_t *bytes);
hipError_t sg_repack(kb_problem *h);
hipError_t sg_power_changed(kb_problem *h);

// Record an error message for kb_last_error(); returns code.
int kb_set_error(int code, const char *msg);

// Reductions recorded inside the iteration chain (every m steps): pass 1
// writes per-block partials of each group of fields, pass 2 sums them in a
// fixed order and appends {step, value_0, value_1, 0} to a device log at
// the index held by a device counter, which it then increments.
struct RedLogArgs {
  const float *f[6];
  int nf, ngroups, square, nb;  // nf fields, split evenly into ngroups sums
  long long n, chunk;           // elements per field, elements per block
  double *partials;             // [ngroups][nb]
  double *log;                  // [cap][4]
  long long *count;
  long long cap, every;
};
constexpr long long kRedLogCap = 4096;
void make_reduce_log(Launch &L1, Launch &L2, const RedLogArgs &a);
RedLogArgs reduce_log_args(const float *const *fields, int nf, int ngroups, int square, long long n, double *partials,
                           double *log, long long *count, long long every);

// Deterministic reductions (enqueued on s; partials has >= reduce_max_blocks doubles).
int reduce_max_blocks();
hipError_t reduce_sum(const float *x, long long n, double *partials, double *result, hipStream_t s);
// Sum (square = 0) or sum of squares (1) over nf <= 6 arrays of n floats
// into *result; partials holds >= reduce_max_blocks doubles.
hipError_t reduce_impl(const float *const *f, int nf, int square, long long n, double *partials, double *result,
                       hipStream_t s);
constexpr long long kReduceNoallocMaxN = 1LL << 40;
hipError_t stream_probe(int nin, int nout, long long n, float *ws, hipStream_t s, int reps, double *seconds);
hipError_t reduce_sumsq(const float *const *fields, int nf, long long n, double *partials, double *result,
                        hipStream_t s);

// ---------------------------------------------------------------------------
// Problem state.
// ---------------------------------------------------------------------------
struct FieldRef {
  float *ptr = nullptr;         // device
  size_t bytes = 0;
  bool host_only = false;       // lives in host memory of the handle
  float *host = nullptr;
};

}  // namespace kb

struct kb_problem {
  int kind = 0;
  int K = 1;                    // kernels per iteration
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  int device = 0;
  unsigned char *ws = nullptr;
  size_t ws_bytes = 0;

  // options
  int builder = 0;              // 0 explicit nodes, 1 stream capture
  int tile = 0;                 // kernel variant (0 = default)
  int tdepth = 1;
  int cache = 1;
  int64_t max_nodes = 65536;
  int graph_update = 0;         // 1: refit cached graphs when node arguments change
  int persistent = 0;           // 1: one cooperative launch per kb_run (many grids)
  int64_t spin_limit = 0;       // polls per barrier wait of that launch (0: automatic)
  double t_update_s = 0;        // host time of the last refit / invalidation
  int64_t n_updated = 0;        // graphs refitted by it

  // heat
  float *Tbuf[2] = {nullptr, nullptr};
  float *P = nullptr;
  int cur = 0;                  // index of the buffer holding the current T
  int64_t nz = 1, ny = 0, nx = 0;
  kb::HeatCoef hk{};
  // multi
  int G = 0;
  kb::GridDesc *grids_d = nullptr;
  int *block_start_d = nullptr;
  int total_blocks = 0;
  kb::GridDesc *grids2_d = nullptr;   // 64 x 32 strip tiling
  int *block_grid_d = nullptr;
  int total_blocks2 = 0;
  kb::GridDesc *grids_tb_d = nullptr;  // temporal-blocking tilings, per (region shape, depth)
  int *block_grid_tb_d = nullptr;
  int tb_start[kb::kMtTilings + 1] = {0};    // first entry of each tiling's block table
  unsigned *grid_bar_d = nullptr;             // persistent kernel's barrier words
  int persist_blocks = 0;                     // resident 256-thread blocks (0: not queried yet)
  int64_t total_cells = 0;
  std::vector<int64_t> grid_shape;
  // skeleton
  float *x = nullptr;
  int64_t n = 0;
  std::vector<float> a, b;
  // fdtd
  int N = 0;
  int pitch = 0;                // FDTD row pitch in floats (multiple of 4)
  float dt = 0.5f;
  float *F[2][6] = {};          // two buffer sets; the current one is F[cur]
  float *g = nullptr; int glen = 0;
  float *probe = nullptr; int pcap = 0;
  long long *step = nullptr;
  unsigned *done = nullptr;           // finished blocks of the running whole-row launch
  long long src = 0;
  int src_ijk[3] = {0, 0, 0};
  // learned surrogate (KB_HEAT2D_SURROGATE)
  kb::SgState *sg = nullptr;
  // reductions
  double *partials = nullptr;   // 2 * reduce_max_blocks doubles
  double *red = nullptr;
  int64_t red_every = 0;        // in-chain reduction every m steps (0: off)
  int64_t step_count = 0;       // steps since red_every was set
  double *redlog = nullptr;     // [kRedLogCap][4]
  long long *redcount = nullptr;

  // graphs: key (b, tdepth, tile, start parity, start step mod red_every)
  std::map<std::tuple<int64_t, int, int, int, int64_t>, hipGraphExec_t> cache_map;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  kb_timing last{};
  bool timed = false;
  int64_t host_steps = 0;
};
