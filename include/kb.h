/*
 * kb.h -- C ABI of libkbatch: iteration-batched graph execution of
 * iterative GPU solvers on one MI355X (gfx950).
 *
 * The library implements the method of "Boosting Performance of Iterative
 * Applications on GPUs: Kernel Batching with CUDA Graphs" (Ekelund,
 * Markidis, Peng, arXiv 2501.09398) with HIP graphs: an iterative solver
 * runs either one launch per kernel per iteration (the baseline loop of
 * Sec. III-A, Listings 1-2) or in iteration batches of b iterations that are
 * unrolled into one static graph, instantiated, uploaded and replayed
 * (Sec. III-A, Listing 3), with the remainder n mod b run per launch (the
 * loop peeling named in Sec. VI).
 *
 * Conventions
 *   - Every entry point returns an int status: 0 = OK, < 0 = error,
 *     > 0 = warning (the call did its work).  kb_last_error() gives the
 *     message of the last failing call on the calling thread.
 *   - No C++ exception crosses this boundary.
 *   - Device memory is owned by the caller: kb_create() receives one
 *     workspace of at least kb_workspace_bytes() bytes (device pointer,
 *     256-byte aligned) and keeps using it until kb_destroy().  The library
 *     allocates no device memory of its own for problem state.
 *   - All device work of a handle is enqueued on the one HIP stream given
 *     to kb_create() (borrowed, never destroyed by the library).  Calls are
 *     asynchronous unless stated otherwise.
 *   - A handle must not be used by two threads at once.
 */
#ifndef KB_H
#define KB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define KB_OK          0
#define KB_EINVAL     -1   /* bad argument (shape, coefficient, field, size) */
#define KB_ENOMEM     -2   /* workspace smaller than kb_workspace_bytes()    */
#define KB_EHIP       -3   /* a HIP runtime call failed; see kb_last_error() */
#define KB_ESTATE     -4   /* call not valid in the handle's current state  */
#define KB_WFALLBACK   1   /* graph build failed; the steps ran per launch  */

/* ---- problems ---------------------------------------------------------- */
/* Each problem is one iterative application of Sec. III-C (or the batched
 * many-grid variant).  shape and coeffs per problem:
 *
 * KB_HEAT2D  (Hotspot-style explicit thermal update, one kernel per step)
 *   shape  = {ny, nx}                 grid rows, columns (>= 1 each)
 *   coeffs = {c, Rx, Ry, Rz, Tamb}    per step, with clamped neighbours:
 *            T' = T + c*(P + (Tn+Ts-2T)/Ry + (Te+Tw-2T)/Rx + (Tamb-T)/Rz)
 *            Requires c*(2/Rx + 2/Ry + 1/Rz) < 1 (monotone update).
 *   fields : KB_F_T (ny*nx float, row-major), KB_F_P (ny*nx float)
 *   initial: T ~ U[323,343), P ~ U[0,1) from the seed.
 *
 * KB_HEAT3D  (Hotspot3D-style layered update, one kernel per step)
 *   shape  = {nz, ny, nx}; coeffs as KB_HEAT2D.  Adds (Tu+Td-2T)/Rz with a
 *            clamped layer index; ambient term on every layer; the power P
 *            is nonzero only in layer z = 0 and stored as one ny*nx plane.
 *            Requires c*(2/Rx + 2/Ry + 3/Rz) < 1.
 *   fields : KB_F_T (nz*ny*nx float, [z][y][x]), KB_F_P (ny*nx float)
 *
 * KB_SKELETON  (the skeleton application: K small element-wise kernels per
 *   iteration; kernel k computes x <- a_k*x + b_k with one rounding)
 *   shape  = {n}                      vector length (>= 1)
 *   coeffs = {K} or {K, a_1..a_K, b_1..b_K}; 1 <= K <= 16.  With K alone the
 *            a_k ~ U[0.9,1), b_k ~ U[-0.01,0.01) come from the seed.
 *   fields : KB_F_X (n float), KB_F_A (K float), KB_F_B (K float)
 *   initial: x ~ U[-1,1).
 *
 * KB_FDTD3D  (FDTD Maxwell solver of a PEC cavity: per step an H update, an
 *   E update and the soft source -- two kernels with the fused H + E step
 *   (default), three with the separate ones)
 *   shape  = {N} or {N, probe_capacity}: cells per edge (4 <= N <= 1024)
 *            and the number of steps of Ez(src) recorded (default 16384).
 *   coeffs = {courant, width, delay} or {courant, width, delay, i, j, k}
 *            dt = courant (dx = 1, eps = mu = 1; needs courant < 1/sqrt(3));
 *            after the E update of absolute step n (counted from 0),
 *            Ez(src) += float(exp(-((n - delay)/width)^2)) (no source for
 *            width <= 0; delay + 10.2*width must stay below 4095 steps).
 *            The source is the Ez node (i, j, k+1/2); it is drawn from the
 *            seed (2 <= i, j <= N-2, 1 <= k <= N-2) unless given, and must
 *            be an interior Ez node (1 <= i, j <= N-1, 0 <= k <= N-1).
 *   fields : KB_F_EX..KB_F_HZ ((N+1)^3 float each, index (k*(N+1)+j)*(N+1)+i),
 *            KB_F_PROBE (probe_capacity float: Ez(src) after step n),
 *            KB_F_STEP (one int64: steps done).
 *   initial: all fields zero.
 *
 * KB_HEAT2D_MULTI  (many independent 2D grids of uneven sizes advanced
 *   together: one kernel per iteration over all grids, an iteration being
 *   one step or, with temporal blocking, KB_OPT_TDEPTH steps; or all steps
 *   in one persistent launch, KB_OPT_PERSISTENT)
 *   shape  = {G, ny_0, nx_0, ny_1, nx_1, ...}; coeffs as KB_HEAT2D.
 *   fields : KB_F_T, KB_F_P as the concatenation of the grids, row-major each.
 *   initial: grid g draws its cells at flat offset sum_{h<g} ny_h*nx_h of the
 *            same streams as KB_HEAT2D.
 */
/*
 * KB_HEAT2D_SURROGATE  (the 2D thermal problem advanced k steps at a time by
 *   a learned surrogate, with the plain stencil as checked fallback)
 *   shape  = {ny, nx} or {ny, nx, train_pixels}: the field (ny, nx >= 32)
 *            and the pixel capacity of one training batch (crops x C x C).
 *   coeffs = {c, Rx, Ry, Rz, Tamb} or {c, Rx, Ry, Rz, Tamb, s, threshold, k}
 *            (defaults s = 0.8, threshold = 1e-3, k = 16; 1 <= k <= 16).
 *   initial: T ~ U[323,343) from the seed; the power map P is U[0,1) plus
 *            1-4 Gaussian hot spots: count 1 + floor(4u), then per spot h
 *            centre row u*ny, centre column u*nx, amplitude 1 + 3u and
 *            width sigma = 4 + 28u, u the draws 0 and 1+4h .. 4+4h of
 *            stream 7; P = float(u_P + sum_h amp exp(-r^2 / (2 sigma^2)))
 *            evaluated in double (the learned part's training inputs).
 *            One iteration is one block of k steps:
 *              y = NN((T-333)/10, (P-0.5)/0.29)  (4 layers of 3x3 conv, 32
 *                  channels, GELU, replicate padding; bf16 operands on the
 *                  matrix cores, float32 accumulation);
 *              T_k = T + s*y  (float32);
 *              residual r = max(r_mean, r_tile) (the mean of T against its
 *                  exact k-step recurrence; four seeded 32x32 tiles against
 *                  the plain stencil), both relative to max|T_k|; tile t
 *                  has its origin at row floor(u*(ny-31)), column
 *                  floor(u'*(nx-31)), u and u' the generator's draws 2t and
 *                  2t+1 of stream 10 of the seed;
 *              if r > threshold the block is redone with k plain steps
 *                  from T (one predicated launch; the graph stays static).
 *            n_steps mod k steps run as plain steps.
 *   fields : KB_F_T, KB_F_P as KB_HEAT2D; KB_F_W (19393 float weights:
 *            W1[32][2][3][3], b1[32], W2[32][32][3][3], b2[32],
 *            W3[32][32][3][3], b3[32], W4[1][32][3][3], b4[1]; zero at
 *            creation = no change); KB_F_SGSTATS (int64[2]: blocks checked,
 *            fallbacks); KB_F_RESID (double[4096]: r of each checked block).
 */
#define KB_HEAT2D        1
#define KB_HEAT3D        2
#define KB_SKELETON      3
#define KB_FDTD3D        4
#define KB_HEAT2D_MULTI  5
#define KB_HEAT2D_SURROGATE 6

/* ---- fields (kb_read / kb_write) --------------------------------------- */
#define KB_F_T      1
#define KB_F_P      2
#define KB_F_X      3
#define KB_F_A      4
#define KB_F_B      5
#define KB_F_EX    10
#define KB_F_EY    11
#define KB_F_EZ    12
#define KB_F_HX    13
#define KB_F_HY    14
#define KB_F_HZ    15
#define KB_F_PROBE 16
#define KB_F_STEP  17   /* int64 count of steps advanced on the device */
#define KB_F_W     20   /* surrogate weights (float32[19393])           */
#define KB_F_SGSTATS 21 /* surrogate blocks checked, fallbacks (int64[2]) */
#define KB_F_RESID 22   /* surrogate residual per checked block (double[4096]) */
#define KB_F_REDLOG 23  /* in-chain reduction log (double[4096][4]), see
                           KB_OPT_REDUCE_EVERY                             */
#define KB_F_REDCOUNT 24 /* entries appended to the log (one int64; it keeps
                           counting past the log's 4096 rows)             */
/* The tape of the last kb_sg_loss_grad / kb_sg_train_step batch of a
 * KB_HEAT2D_SURROGATE problem (read only; KB_EINVAL before the first batch
 * and for kb_write).  m = ncrop*crop*crop pixels in crop-major, row-major
 * order; channels contiguous per pixel:
 *   KB_F_SG_X        bf16 bits (uint16) [m][2]   network input (t, p)
 *   KB_F_SG_A1..A3   bf16 bits (uint16) [m][32]  hidden activations
 *   KB_F_SG_Z1..Z3   float [m][32]               pre-activations
 *   KB_F_SG_Y        float [m]                   network output y
 *   KB_F_SG_TGT      float [m]                   target (T16 - T0)/s
 *   KB_F_SG_G4       float [m]                   dL/dy
 *   KB_F_SG_G1..G3   float [m][32]               dL/dz of the hidden layers
 *   KB_F_SG_GRAD     float [19393]               dL/dw (canonical order)
 * So each convolution of the GPU path can be checked on its own operands. */
#define KB_F_SG_X    30
#define KB_F_SG_A1   31
#define KB_F_SG_A2   32
#define KB_F_SG_A3   33
#define KB_F_SG_Z1   34
#define KB_F_SG_Z2   35
#define KB_F_SG_Z3   36
#define KB_F_SG_Y    37
#define KB_F_SG_TGT  38
#define KB_F_SG_G4   39
#define KB_F_SG_G1   40
#define KB_F_SG_G2   41
#define KB_F_SG_G3   42
#define KB_F_SG_GRAD 43

/* ---- options (kb_set_option) ------------------------------------------- */
/* KB_OPT_BUILDER: how a batch graph is built.
 *   0 = explicit kernel nodes (hipGraphAddKernelNode chain, Listing 3)
 *   1 = stream capture of the per-launch loop (Sec. II)                   */
#define KB_OPT_BUILDER   1
/* KB_OPT_TILE: kernel variant (0 = default for the shape).  Every variant
 * of a problem produces the same bits.
 *   KB_HEAT2D: 1 = one thread per cell (64x4 blocks);
 *              2..7 = LDS halo tile with temporal blocking (KB_OPT_TDEPTH),
 *                     tiles 64x4, 64x8, 64x16, 32x8, 16x16, 32x4;
 *              8..12 = float4 rows, a wave walking 1, 2, 4, 8, 16 rows;
 *              13, 14 = 1 and 2 rows with streaming (non-temporal) stores
 *                     and loads of P
 *                     (8..14 need nx % 4 == 0);
 *              15, 16, 17 = temporal blocking over 16x16 tiles with the rows
 *                     of each region column in registers, 4, 2 or 1 per
 *                     thread (KB_OPT_TDEPTH 1..8);
 *              18, 19 = temporal blocking over regions of 64 columns x 64
 *                     or 128 rows, a wave holding 16 rows of one column
 *                     per lane in registers (KB_OPT_TDEPTH 1..8; the
 *                     many-grid problem's variants 3 and 4 on one grid);
 *              20, 21 = the same over regions of 128 columns x 64 or 128
 *                     rows, two columns per lane (KB_OPT_TDEPTH 1..8);
 *              22, 23 = the register strips of 15..17 over 32x32 tiles in
 *                     regions of up to 64 x 64 cells, 4 or 8 rows per
 *                     thread (KB_OPT_TDEPTH 1..16).
 *              Default: 13 if nx % 4 == 0 and ny*nx >= 2^20, else 1.
 *   KB_HEAT3D: 1 = one thread per column; float4 rows (nx % 4 == 0):
 *              2 = plain, 3 = next layer prefetched, 4 = prefetched with
 *              streaming stores and P loads; 5 = temporal blocking (KB_OPT_TDEPTH
 *              steps per launch, 1..6; nz <= 8); 6, 7, 8 = each wave
 *              covers 2, 4, 8 rows with their neighbour rows in registers,
 *              streaming stores and P loads (nx % 4 == 0); 9, 10 = 2, 4 rows with the
 *              layer after next loaded one layer ahead; 11 = temporal
 *              blocking with every layer of a region column's rows in
 *              registers (KB_OPT_TDEPTH 1..8; nz <= 8).  Default: 9 if nx % 4 == 0
 *              and ny*nx >= 2^20, else 1.
 *   KB_SKELETON: 1 = 4 elements per thread (default), 2 = 1, 3 = 8.
 *   KB_FDTD3D: separate H and E kernels (3 kernels per iteration with the
 *              source): 1 = one thread per cell, 2 = float4 rows, 3 / 4 =
 *              float4 rows, each thread walking 8 / 16 planes in k;
 *              fused H + E step (2 kernels per iteration): 5 = float4 rows,
 *              one plane per thread, 6 = walking 8 planes, 7 = as 5 with
 *              streaming (non-temporal) stores; 8 = two steps per launch
 *              with KB_OPT_TDEPTH 2 (blocks march along k, the intermediate
 *              E and H rows shared through LDS; streaming stores when the
 *              sets exceed 256 MiB), the fused step with depth 1 (and for
 *              the last step of an odd count); 9, 10 = as 8 with a wave
 *              holding a whole row, four nodes per lane (N <= 256, else as
 *              8; 9: 16 rows per block, 10: 12 rows per block with the
 *              next plane's operands loaded ahead; one kernel per two-step
 *              iteration, which also advances the step counter); with
 *              KB_OPT_TDEPTH 3, 9 and 10 take three steps per launch (12
 *              rows per block, 7 of them output; two nodes per lane up to
 *              N = 128).  Default: 7 when the two
 *              field sets exceed 256 MiB (N >= 176), else 5.  The
 *              fused step reads one set of six fields and writes the other
 *              (48 instead of 72 bytes per node-step), so the state
 *              alternates between two sets like the stencils' ping-pong
 *              buffers; every variant continues from the current set.
 *   KB_HEAT2D_MULTI: 1 = one thread per cell (64x4 tiles, grid found by
 *              binary search); 2 = each wave walks 8 rows of 64 columns
 *              with the neighbour rows in registers (64x32 tiles, grid from
 *              a block table); 3 (default), 4 = temporal blocking
 *              (KB_OPT_TDEPTH steps per launch, 1..8) over regions of 64
 *              columns x 64 (3) or 128 (4) rows around output tiles of
 *              (64-2t) x (64-2t or 128-2t) cells, each region column's
 *              rows in registers; 5, 6 = the same over regions of 128
 *              columns x 64 (5) or 128 (6) rows, two columns per lane.
 *   KB_HEAT2D_SURROGATE: 1 = fused network, all activations in LDS, 3
 *              kernels per block (default); 2 = one kernel per layer with
 *              activations in HBM, 8 kernels per block.  The two agree to
 *              float32 rounding of the last layer's sum, not bit for bit. */
#define KB_OPT_TILE      2
/* KB_OPT_TDEPTH: temporal-blocking depth t >= 1: one launch of a
 *   temporal-blocking variant advances t steps (KB_HEAT2D LDS tile 1..16,
 *   register strips 15..17 1..8, register regions 18..21 1..8, register
 *   strips 22, 23 1..16; KB_HEAT3D variant 5 1..6, variant 11 1..8;
 *   KB_HEAT2D_MULTI variants 3..6 1..8; KB_FDTD3D variants 8..10 1..2 and
 *   variants 9, 10 also 3 (N <= 256), the option taking 1..3 for every
 *   cavity variant; a launch whose variant does not allow t fails with
 *   KB_EINVAL).  Other variants ignore it.  kb_run advances
 *   floor(n_steps / t) iterations of t steps, then n_steps mod t single
 *   steps per launch.                                                      */
#define KB_OPT_TDEPTH    3
/* KB_OPT_GRAPH_CACHE: 1 = keep instantiated batch graphs between kb_run
 *   calls (default), 0 = rebuild every call (each call then pays T_C).    */
#define KB_OPT_GRAPH_CACHE 4
/* KB_OPT_MAX_NODES: refuse graphs with more kernel nodes (default 65536). */
#define KB_OPT_MAX_NODES 5
/* KB_OPT_REDUCE_EVERY: m >= 1 appends a deterministic reduction of the
 *   state after every m-th step to the iteration chain itself (two extra
 *   kernels, recorded as graph nodes inside batch graphs, so a replayed
 *   graph reduces with no host involvement): the sum of T (heat problems,
 *   all grids together for KB_HEAT2D_MULTI), the sum of x (KB_SKELETON), or
 *   E.E and H.H over the six FDTD fields.  Entry e of KB_F_REDLOG is
 *   {(e+1)*m, value, second value or 0, 0}; KB_F_REDCOUNT counts entries.
 *   Setting the option (also to 0 = off, the default) restarts the step
 *   count and empties the log.  With temporal blocking (t steps per
 *   iteration) m, n_steps and the steps run since the option was set must
 *   be multiples of t, so that every reduction point ends an iteration;
 *   not for KB_HEAT2D_SURROGATE.  Each graph batch is built for
 *   its start phase (steps since the last reduction point), so b need not
 *   divide m; at most 64 distinct batch graphs per kb_run.  Results are
 *   bitwise independent of b and of the builder.                          */
#define KB_OPT_REDUCE_EVERY 6
/* KB_OPT_GRAPH_UPDATE: what a kb_write of arguments that are baked into
 *   graph nodes (KB_F_A / KB_F_B of KB_SKELETON) does to the cached batch
 *   graphs: 0 = drop them (the next kb_run rebuilds and pays T_C again;
 *   default), 1 = refit each in place with hipGraphExecUpdate (the graph is
 *   recorded again with the new arguments but not instantiated; a graph the
 *   runtime refuses to update is dropped).  Either way the results are the
 *   same bits.  The paper notes that graphs are hard to change once built
 *   (Sec. II); this measures what an in-place update costs on MI355X.     */
#define KB_OPT_GRAPH_UPDATE 7
/* KB_OPT_PERSISTENT (KB_HEAT2D_MULTI only): 1 = kb_run advances all grids
 *   in ONE cooperative launch of a persistent kernel (every block resident)
 *   instead of per-launch iterations or graph batches: super-steps of
 *   KB_OPT_TDEPTH steps over the 64 x 64-region temporal-blocking tiles
 *   (variant 3's), each ended by a grid-wide barrier, and one super-step
 *   of n_steps mod t steps at the end.  batch_b is ignored; the kernel
 *   variant option is not consulted.  The run is synchronous (kb_run waits
 *   for the launch and checks the barrier's error flag: KB_EHIP if a
 *   barrier wait timed out).  Not with KB_OPT_REDUCE_EVERY.  Same bits as
 *   every other variant.  0 = off (default).  The alternative to graphs
 *   that the paper sets against them (Sec. V): no launch per step at all. */
#define KB_OPT_PERSISTENT 8
/* KB_OPT_SPIN_LIMIT: polls a grid-barrier wait of the persistent kernel
 *   makes before it gives up (raising the error flag that makes kb_run
 *   return KB_EHIP; no block waits after that, so the launch always ends).
 *   0 = automatic (about a second, more for very large super-steps).     */
#define KB_OPT_SPIN_LIMIT 9

typedef struct kb_problem kb_problem;

/* Timing of the most recent kb_run() (Sec. III-B, Eqs. 1-2): the host wall
 * time spent building, instantiating and uploading graphs (T_C, including
 * the upload, as in Sec. IV-A), and the device time of the launches
 * measured with HIP events around them (T_E).                             */
typedef struct kb_timing {
    double t_create_s;        /* T_C of graphs built by this call          */
    double t_exec_s;          /* T_E: events around all launches of the call */
    int64_t n_graph_launches; /* graph launches                            */
    int64_t n_nodes;          /* kernel nodes per batch graph (K*b)       */
    int64_t n_peeled;         /* iterations run per launch (remainder)     */
    int64_t n_kernel_launches;/* individual kernel launches                */
    int64_t n_graphs_built;   /* graphs built by this call (cache misses)  */
    int64_t graph_mem_bytes;  /* drop of the device's free memory across
                                 building, instantiating and uploading
                                 those graphs (hipMemGetInfo; the graphs'
                                 own footprint on an otherwise idle device,
                                 the quantity of the paper's Fig. 2 bars) */
    double t_update_s;        /* host time of the last kb_write that changed
                                 arguments baked into graph nodes (skeleton
                                 a_k, b_k): refitting (KB_OPT_GRAPH_UPDATE=1)
                                 or dropping the cached graphs            */
    int64_t n_graphs_updated; /* graphs refitted in place by that write    */
} kb_timing;

/* Device bytes kb_create() needs for this problem and shape; 0 if the
 * problem or shape is invalid.  Pure; no HIP call.                         */
size_t kb_workspace_bytes(int problem, const int64_t *shape, int ndim);

/* Create a problem on the current HIP device.
 *   workspace: device pointer of >= kb_workspace_bytes() bytes, 256-B
 *              aligned, owned by the caller and kept alive until destroy.
 *   stream   : hipStream_t (as void*) to enqueue on; NULL = null stream.
 *   Fills the initial state on the device from seed (counter-based
 *   SplitMix64, one draw per cell), enqueued on the stream.
 * Errors: KB_EINVAL (problem, shape, coefficients, unstable c or dt),
 *         KB_ENOMEM (workspace too small or misaligned), KB_EHIP.          */
int kb_create(int problem, const int64_t *shape, int ndim,
              const double *coeffs, int ncoeffs, uint64_t seed,
              void *workspace, size_t ws_bytes, void *stream,
              kb_problem **out);

/* Set an option (KB_OPT_*).  Invalidates cached graphs when it changes
 * the kernels.  KB_EINVAL for an unknown option or value.                 */
int kb_set_option(kb_problem *h, int option, int64_t value);

/* Advance the state by exactly n_steps time steps (Sec. III-A).
 *   batch_b == 0 : per-launch loop, one launch per kernel per iteration
 *                  (Listings 1-2).
 *   batch_b >= 1 : floor(n_iter / b) launches of a graph that unrolls b
 *                  iterations as a linear chain of kernel nodes (Listing 3),
 *                  then n_iter mod b iterations per launch (loop peeling,
 *                  Sec. VI).  An iteration is the problem's K kernels;
 *                  with temporal depth t, one iteration advances t steps
 *                  and n_steps mod t steps run as depth-1 iterations.
 *   Graphs are built on first use per (b, t, buffer parity) and cached.
 *   The result is bit-identical for every b (the same kernels run in the
 *   same order on the same arguments).
 * Errors: KB_EINVAL (n_steps < 0, batch_b < 0, K*b > max nodes), KB_EHIP.
 * Warning: KB_WFALLBACK if a graph could not be built and the iterations
 *          ran per launch instead.                                        */
int kb_run(kb_problem *h, int64_t n_steps, int64_t batch_b);

/* Copy one field out: the state an iterative application has after its
 * loop of kernel iterations (Sec. III-A, the iteration loop of Listings
 * 1-2; the applications' outputs of Sec. III-C).  Synchronises the stream
 * first.  dst is host memory (dst_on_device = 0) or device memory (1);
 * bytes must equal the field's size.  Errors: KB_EINVAL (field or size),
 * KB_EHIP.                                                                 */
int kb_read(kb_problem *h, int field, void *dst, size_t bytes,
            int dst_on_device);

/* Overwrite one field: the application's input state before its loop
 * (Sec. III-A; prescribed initial states, and resuming a loop split across
 * kb_run calls, which must equal one run of the total count).  Synchronises
 * the stream after the copy.  Same errors as kb_read.                      */
int kb_write(kb_problem *h, int field, const void *src, size_t bytes,
             int src_on_device);

/* Deterministic device reduction of the current state (fixed-order wave64
 * tree, double accumulation across blocks), synchronous: the checks an
 * application makes of its state (mean T against the heat equation's
 * closed-form mean, the FDTD cavity's discrete energy); the paper's
 * applications check their results, its method does not define them.
 *   KB_HEAT2D/3D/MULTI: out[0] = sum of T
 *   KB_SKELETON       : out[0] = sum of x
 *   KB_FDTD3D         : out[0] = sum of E.E, out[1] = sum of H.H
 * Errors: KB_EINVAL, KB_EHIP.                                              */
int kb_reduce(kb_problem *h, double *out, int nout);

/* kb_reduce without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same deterministic two-pass sum (the same kernels,
 * chunks and summation order as kb_reduce, so the same bits for the same n)
 * over caller arrays, with the per-block partials in a static device array
 * of the library (1024 doubles = 8 KiB per GPU, held until the process
 * ends).
 *   x      : host array of nx (1..6) device pointers, each to n floats
 *   n      : elements per array, 0 <= n <= 2^40
 *   square : 0 = sum of all elements, 1 = sum of their squares
 *   out    : device pointer to one double, written on the stream
 *   stream : hipStream_t (as void*); work is enqueued, not waited for
 * Allocates nothing: no hipMalloc, no hipFree, no memset.  The first call on
 * a device resolves the static array's address there (make it outside a
 * graph capture).  Calls on one GPU share its array: calls whose work
 * overlaps on that GPU (other streams, other threads) race and must be
 * ordered by the caller.  The current device must be the stream's device.
 * Errors: KB_EINVAL (counts, n, null pointers), KB_EHIP.                  */
int kb_reduce_noalloc(const float *const *x, int nx, int64_t n, int square, double *out, void *stream);

/* Timing of the last kb_run() (synchronises the stream).                   */
int kb_last_timing(kb_problem *h, kb_timing *out);

/* Surrogate training (KB_HEAT2D_SURROGATE created with train_pixels > 0).
 * The batch is ncrop crops of crop x crop pixels (crop a multiple of 64,
 * ncrop*crop^2 <= train_pixels, ncrop <= 1024) cut from stored fields:
 *   T0, P, T16 : device float32 [nfield][Hf][Wf]: start state, power map,
 *                and the state after k plain steps (the target is
 *                (T16 - T0)/s);
 *   crops      : host int32 [ncrop][3] = {field, y0, x0}.
 * The loss is the mean over the batch's pixels of (y - target)^2; the
 * gradient covers all 19393 weights (float32 accumulation of bf16
 * products; per-block partial sums in a fixed order, so it is
 * deterministic).  Synchronous.
 * kb_sg_loss_grad  : loss (host, may be NULL) and gradient (host float
 *                    [19393], may be NULL); the weights are unchanged.
 * kb_sg_train_step : one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 *                    bias-corrected with the handle's step count) at
 *                    learning rate lr; loss (may be NULL) is the batch loss
 *                    before the step.
 * Errors: KB_EINVAL (not a surrogate, crop outside its field, batch too
 *         large), KB_EHIP.                                                 */
int kb_sg_loss_grad(kb_problem *h, const float *T0, const float *P, const float *T16, int nfield, int Hf,
                    int Wf, const int *crops, int ncrop, int crop, double *loss, float *grad);
int kb_sg_train_step(kb_problem *h, const float *T0, const float *P, const float *T16, int nfield, int Hf,
                     int Wf, const int *crops, int ncrop, int crop, double lr, double *loss);

/* Number of kernels per iteration (K) of the problem, or < 0 on error.    */
int kb_kernels_per_iter(const kb_problem *h);

/* Destroy graphs, events and the handle; the workspace stays the caller's
 * (the end of the application, after which its graphs are destroyed, as in
 * the measurement of a graph's memory before that point, Sec. III-C).
 * Synchronises the stream.  NULL is accepted.                              */
int kb_destroy(kb_problem *h);

/* Message of the last failing call on this thread ("" if none).  Valid
 * until the next kb_* call on the same thread.                             */
const char *kb_last_error(void);

/* Streaming calibration (a measurement helper, not part of a solver): time
 * one kernel that reads nin arrays and writes nout arrays of n floats each
 * (1 <= nin, nout <= 8; n a multiple of 4), element-wise, float4 per thread
 * -- the access pattern of a stencil or FDTD kernel with that many
 * concurrent HBM streams, with no reuse and no arithmetic to speak of.  It
 * gives the DRAM throughput attainable for a kernel's stream mix, against
 * which the kernel's own throughput can be read.
 *   workspace: device pointer of >= (nin + nout) * n * 4 bytes, 256-B
 *              aligned (the caller's; contents overwritten); array k
 *              starts at byte k * n * 4.
 *   stream   : hipStream_t to run on (NULL = default stream).
 *   reps     : timed launches after one untimed launch.
 *   seconds  : out, mean seconds per launch (HIP events; synchronises).
 * Returns KB_OK, KB_EINVAL (bad counts, n, size or alignment), KB_EHIP.   */
int kb_stream_probe(int nin, int nout, int64_t n, void *workspace, size_t ws_bytes, void *stream, int reps,
                    double *seconds);

/* ABI version of this header (increments on incompatible change).         */
int kb_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KB_H */
