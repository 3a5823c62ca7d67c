// Internal declarations shared by the planner's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdp.h"

namespace mdpk {

constexpr int kBlock = 256;          // threads per workgroup of every build / VI kernel
constexpr int kMaxA = MDP_MAX_ACTIONS;

// Device-side bookkeeping at the start of the build scratch.
struct BuildState {
  unsigned long long n_escape;
  unsigned long long n_near;
  unsigned long long samples;
  long long running_nnz;  // nonzeros of all slabs finished so far
  mdp_build_stats out;    // filled by the finalize kernel, copied to the host
  long long pad[8];
};

// Problem-wide parameters of the build kernels (passed by value).
struct BuildParams {
  const float *ubar, *vbar, *phiu, *phiv, *mu, *gbar;
  const uint8_t *mask;
  float *reward;            // [nmiss][rows]
  int64_t rows;
  int nx, ny, nt, nc, na, nr, K;
  int hx, hy, W, nsg;
  int nbins;                // histogram bins: nsg, plus the swept-path DEAD bin
  int ti, tj;               // target cell
  int mean_tstride;         // nc if the mean varies in time, else 0 (elements)
  int64_t mode_tstride;     // K*nc if the modes vary in time, else 0
  int cells_per_tile, tiles_per_layer, rch;
  int row_lanes;            // lanes that own a (cell, action) row: 256, 128 or 64
  int hw;                   // LDS words per sub-grid bin (row_lanes, or half with 16-bit counters)
  int nmiss, miss[3];
  int n_head, n_speed;
  float lam_x, lam_y, eps_x, eps_y;
  float usafe, vsafe;       // |u| <= usafe and |v| <= vsafe rule out any escape
  double dt, r_term, r_out, c_f, c_r, f_max;
  const float *tab;         // device [2][kMaxA]: Hx then Hy (cell units per step)
  // Paired landing loop (16-bit counters): the actions form n_pairs = N_a / 2
  // pairs, the first n_real_pairs of them with bitwise-equal Hx (so both rows
  // of the pair land in the same column); pair q is actions pair_a[2q] (low
  // counter half) and pair_a[2q + 1] (high half); row_pair[a] = q << 1 | half.
  int paired, n_real_pairs;
  uint8_t pair_a[kMaxA];
  uint8_t row_pair[kMaxA];
};

// Host-side action tables, copied to the device by a one-thread-per-entry kernel.
struct ActionTables {
  float hx[kMaxA], hy[kMaxA];
};

struct ModelOut {
  int64_t *row_ptr;
  int32_t *col;
  uint16_t *cnt;
  int64_t capacity;
};

// Per-pass parameters: one pass covers decision layers [t0, t0 + nlayers).
struct SlabParams {
  int t0, nlayers;
  int64_t row0;             // first global row of the pass
  uint32_t *row_nnz;        // [pass rows]
  uint32_t *row_off;        // [pass rows] offset of the row inside its workgroup's block
  uint32_t *wg_nnz;         // [pass workgroups]
  int64_t *wg_off;          // [pass workgroups] global offset of the block
  uint64_t *stage;          // [pass workgroups][wg_cap] packed (col, cnt)
  int64_t wg_cap;
  BuildState *st;
};

// One problem of a batch (device-resident descriptor, see batch launchers).
struct BatchBuildDesc {
  BuildParams P;             // P.tab points at this problem's action tables
  BuildState *st;            // this problem's bookkeeping
  uint32_t *row_nnz;         // [rows]
  uint32_t *row_off;         // [rows] offset of the row inside its tile's block
  uint32_t *item_total;      // [n_items] entries of tile item (layer, tile)
  int64_t *item_base;        // [n_items] pool slot of the item (-1: did not fit)
  int64_t *item_off;         // [n_items] global CSR offset of the item
  ModelOut M;
  int64_t n_items;           // nt * tiles_per_layer
  int near_asked;
  int pad;
};

// A batched build runs one persistent launch per group of problems that share
// the kernel variant (mode bound, near-edge counting) and occupancy; each group
// has its own work counter.
constexpr int kMaxBuildGroups = 32;
constexpr int kMaxBuildLaunches = 256;  // work counters of one batched build (groups, or their chunks)

// Work item of the persistent batched build: problem, layer, tile.
struct BatchItem {
  int inst, t, tile, pad;
};

// Swept-path obstacle test (MDP_FLAG_SWEPT_PATH): does the straight step from
// the centre of cell (ci, cj) to the landing point (X, Y), in cell units,
// enter an obstacle cell of mask layer `m1` (the layer at t+1) other than the
// source cell? Each candidate cell of the segment's bounding box is tested
// against the open unit square by separating axes (x, y, the segment's
// normal); with fp32 landing coordinates every difference and product is exact
// in fp64, so the outcome is exact.
__device__ inline bool segment_meets_cell(double x0, double y0, double x1, double y1, int a, int b)
{
  const double lx = fmin(x0, x1), hx = fmax(x0, x1), ly = fmin(y0, y1), hy = fmax(y0, y1);
  if (!(lx < (double)a + 1.0 && hx > (double)a && ly < (double)b + 1.0 && hy > (double)b)) return false;
  const double dx = x1 - x0, dy = y1 - y0;
  const double f00 = dx * ((double)b - y0) - dy * ((double)a - x0);
  const double f10 = dx * ((double)b - y0) - dy * ((double)(a + 1) - x0);
  const double f01 = dx * ((double)(b + 1) - y0) - dy * ((double)a - x0);
  const double f11 = dx * ((double)(b + 1) - y0) - dy * ((double)(a + 1) - x0);
  return fmin(fmin(f00, f10), fmin(f01, f11)) < 0.0 && fmax(fmax(f00, f10), fmax(f01, f11)) > 0.0;
}

__device__ inline bool swept_blocked(const uint8_t *m1, int nx, int ny, int ci, int cj, int ix, int iy, float X,
                                     float Y)
{
  const double x0 = (double)ci + 0.5, y0 = (double)cj + 0.5, x1 = (double)X, y1 = (double)Y;
  const int a0 = max(min(ci, ix), 0), a1 = min(max(ci, ix), nx - 1);
  const int b0 = max(min(cj, iy), 0), b1 = min(max(cj, iy), ny - 1);
  bool hit = false;
  for (int b = b0; b <= b1; ++b)
    for (int a = a0; a <= a1; ++a)
      if (!(a == ci && b == cj) && m1[(size_t)b * nx + a] != 0 && segment_meets_cell(x0, y0, x1, y1, a, b)) hit = true;
  return hit;
}

// Copy of an entry of a device table that no kernel writes while it is read,
// fetched through the constant address space: at a wave-uniform address the
// words arrive by scalar loads instead of occupying vector registers.
template <typename T>
__device__ inline T load_const(const T *p)
{
  static_assert(sizeof(T) % 4 == 0, "word-sized table entries");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const cword *src = (const cword *)(uintptr_t)p;
  T out;
  uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

// Launchers (return hipError_t of the launch)
hipError_t launch_fill_tab(const ActionTables &T, float *tab, hipStream_t s);
hipError_t launch_build_init(BuildState *st, hipStream_t s);
// Build bookkeeping for a rebuild of the layers from row `row0` on: entries
// before it are kept, so the running entry count starts at row_ptr[row0].
hipError_t launch_build_init_from(BuildState *st, const int64_t *row_ptr_row0, hipStream_t s);
hipError_t launch_build_slab(const BuildParams &P, const SlabParams &S, int kmax, bool pack16,
                             bool near, bool swept, size_t lds_bytes, hipStream_t s);
hipError_t launch_scan_wg(const SlabParams &S, int n_wg, int64_t *row_ptr_end, hipStream_t s);
hipError_t launch_copy(const BuildParams &P, const SlabParams &S, const ModelOut &M, int n_wg,
                       hipStream_t s);
hipError_t launch_build_finalize(BuildState *st, int64_t capacity, int n_slabs, int near_asked,
                                 hipStream_t s);
hipError_t launch_escape_only(const BuildParams &P, BuildState *st, hipStream_t s);
hipError_t launch_batch_build_init(BatchBuildDesc *D, int n, unsigned int *counter,
                                   unsigned long long *pool_top, hipStream_t s);
hipError_t launch_batch_build(const BatchBuildDesc *D, const BatchItem *items, int n_items,
                              unsigned int *counter, uint64_t *pool, unsigned long long *pool_top,
                              int64_t pool_cap, int kmax, bool near, size_t lds, int grid, hipStream_t s);
hipError_t batch_build_occupancy(int kmax, bool near, size_t lds, int *blocks_per_cu);
hipError_t launch_batch_scan(BatchBuildDesc *D, int n, hipStream_t s);
hipError_t launch_batch_copy(const BatchBuildDesc *D, const BatchItem *items, int n_items, const uint64_t *pool,
                             hipStream_t s);
hipError_t launch_batch_finalize(BatchBuildDesc *D, int n, mdp_build_stats *out, hipStream_t s);
hipError_t launch_max_speed(const BuildParams &P, unsigned int *umax_bits, hipStream_t s);

// Value iteration / policy
struct VIState {
  unsigned long long res_bits;  // running max of |v_new - v_old| (bits of a non-negative double)
  unsigned int wg_count;
  int done;
  int sweeps;
  int status;
  double last_res;
  long long pad[4];
};

struct VIParams {
  const int64_t *row_ptr;
  const int32_t *col;
  const uint16_t *cnt;
  const float *R;           // reward block of the mission
  const uint32_t *ent;      // packed entries (window index << 16 | cnt), or nullptr (fused sweep only)
  const uint16_t *roff;     // with ent: each row's first entry relative to its block's first entry
  int64_t cap;              // length of col / cnt (and ent)
  int64_t ns;
  int na, nx, ny, nc, nt, hy, hx;
  int narrow;               // packed entries: blocks inside one grid row stage only the columns they reach
  int states_per_wg;        // S: cells of one layer per block, S * na <= 2 * kBlock rows
  int blocks_per_layer;     // ceil(nc / S)
  int64_t n_blocks;         // nt * blocks_per_layer
  int win_rows;             // grid rows of the staged window of v(t + 1); 0: gather from memory
  int max_row;              // most entries a row can hold, min(N_sg, n_real)
  int n_wg;                 // launched workgroups
  int t_lo;                 // first layer a sweep recomputes (0 but for mdp_value_iterate_layers)
  double inv_nr, tol;
  VIState *st;
};

// LDS of the sweep / policy kernels, in doubles: the staged products of one
// chunk of the block's entries (Q of the block's rows reuses it once every row
// sum is done), the wave maxima; then (batched kernels) per-problem residuals,
// block starts and sweep states; then the window of v(t + 1).
constexpr int kViRows = 2 * kBlock;
constexpr int kViChunk = 2048;                         // entries staged per round (>= kViRows)
constexpr int kViProd = 0;
constexpr int kViQ = 0;                                // aliases the products
constexpr int kViWmax = kViProd + kViChunk;
constexpr int kViFixed = kViWmax + 8;
constexpr int kViWinPerThread = 8;                             // window values a thread stages
constexpr size_t kViWinBudget = (size_t)kViWinPerThread * kBlock * 8;  // bytes of the v window at most

// Grid rows the v window of a block needs (rows spanned by S cells plus hy on
// each side), or 0 when it would not fit the budget.
inline int vi_window_rows(int nx, int ny, int hy, int S)
{
  int rows = (S - 1) / nx + 2 + 2 * hy;
  if (rows > ny) rows = ny;
  return (size_t)rows * nx * 8 <= kViWinBudget ? rows : 0;
}

// The window of v(t + 1) a block of cells [c0, c0 + nst) of layer t stages:
// grid rows [j_first - hy, j_last + hy] (clipped) of layer t + 1, whole rows,
// or with `narrow` and a block inside one grid row only the columns
// [i_first - hx, i_last + hx] (clipped). Value (row r, column k) of the
// window sits at r * cols + k; base is the state index of its first value.
// (The packed entries use narrow windows when the reachable columns are at
// most a quarter of a grid row, VIParams::narrow; a per-row copy of a few
// columns costs more than a contiguous copy of whole rows otherwise.)
struct BlockWin {
  int64_t base;
  int rows, cols;
};

__host__ __device__ inline BlockWin block_window(const VIParams &P, int t, int c0, int nst, bool narrow)
{
  const int j0 = c0 / P.nx, j1 = (c0 + nst - 1) / P.nx;
  const int jw0 = j0 - P.hy > 0 ? j0 - P.hy : 0;
  const int jw1 = j1 + P.hy < P.ny - 1 ? j1 + P.hy : P.ny - 1;
  int iw0 = 0, cols = P.nx;
  if (narrow && j0 == j1) {
    const int i0 = c0 - j0 * P.nx, i1 = c0 + nst - 1 - j0 * P.nx;
    iw0 = i0 - P.hx > 0 ? i0 - P.hx : 0;
    const int iw1 = i1 + P.hx < P.nx - 1 ? i1 + P.hx : P.nx - 1;
    cols = iw1 - iw0 + 1;
  }
  return BlockWin{(int64_t)(t + 1) * P.nc + (int64_t)jw0 * P.nx + iw0, jw1 - jw0 + 1, cols};
}

// Layers a sweep recomputes when `sweeps` sweeps of the solve are behind it:
// layers t >= nt - sweeps + 1 are final in both value buffers.
__host__ __device__ inline int vi_active_layers(int nt, int sweeps)
{
  const int a = nt - sweeps + 1;
  return a < 0 ? 0 : (a > nt ? nt : a);
}

// One problem of a batched solve (device-resident descriptor).
struct BatchVIDesc {
  VIParams P;         // P.st points at this problem's sweep state
  VIState *st;
  double *v, *v_alt;  // values (caller) and the second buffer (scratch)
  int32_t *pi;        // policy (caller)
  int64_t pad;
};

constexpr int kMaxBatch = 1024;  // problems per batch

// Mode terms a build kernel is compiled for: K rounded up to even (2..16);
// the terms past K have zero coefficients and leave the sums unchanged.
inline int mode_bound(int k) { return k <= 2 ? 2 : (k >= 16 ? 16 : (k + 1) & ~1); }

// Missions of one model solved together (every descriptor has the same CSR
// and shape; rewards, values and sweep states differ). Passed by value.
constexpr int kMaxMissions = 3;
struct MultiVI {
  BatchVIDesc d[kMaxMissions];
  int m;
  int pad;
};

hipError_t launch_vi_init(VIState *st, int n, hipStream_t s);
// One sweep over layers [0, t_hi) (later layers are final and already in both
// buffers) and its close; returns the grid used.
hipError_t launch_vi_sweep(const VIParams &P, const double *vin, double *vout, int t_hi, double *wg_res,
                           hipStream_t s);
hipError_t launch_vi_sweep_batched(const BatchVIDesc *D, int n, const int64_t *block_start, double *wg_res,
                                   int grid, size_t win_bytes, hipStream_t s);
hipError_t launch_vi_reset_batched(const BatchVIDesc *D, int n, hipStream_t s);
// One fused sweep of every mission of V over layers [0, t_hi) and its close.
hipError_t launch_vi_sweep_missions(const MultiVI &V, int t_hi, double *wg_res, double tol, hipStream_t s);
hipError_t launch_vi_finish_missions(const MultiVI &V, mdp_vi_stats *out, hipStream_t s);
hipError_t launch_vi_status_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out, hipStream_t s);
hipError_t launch_vi_close_batched(const BatchVIDesc *D, int n, int grid, const double *wg_res, double tol,
                                   hipStream_t s);
hipError_t launch_vi_finish_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out, hipStream_t s);
hipError_t launch_policy_batched(const BatchVIDesc *D, int n, const int64_t *block_start, int grid,
                                 size_t win_bytes, hipStream_t s);
hipError_t launch_vi_finish(const VIParams &P, double *v, const double *v_alt, mdp_vi_stats *dev_stats,
                            hipStream_t s);
hipError_t launch_policy(const VIParams &P, const double *v, int32_t *pi, hipStream_t s);
// The packed entries of the fused sweep for layers [t_lo, nt) of a built
// model (P with win_rows > 0): ent[e] = (window index << 16) | cnt, 0xFFFF for
// a sink, and roff[row] = row_ptr[row] - row_ptr[first row of the row's block].
hipError_t launch_compact(const VIParams &P, uint32_t *ent, uint16_t *roff, int t_lo, hipStream_t s);

// Policy rollouts (rollout.hip): one lane per realization.
struct RollParams {
  const float *ubar, *vbar, *phiu, *phiv, *mu, *gbar;
  const uint8_t *mask;
  const int32_t *pi;        // [nt][ny][nx]
  int32_t *traj;            // [nt + 1][n_real] or nullptr
  mdp_rollout_path *paths;  // [n_real]
  int nx, ny, nt, nc, nr, K, na;
  int si, sj, ti, tj;
  int mean_tstride;         // elements
  int64_t mode_tstride;     // elements
  float lam_x, lam_y;
  int swept;                // MDP_FLAG_SWEPT_PATH
  double dt, r_term, r_out, c_f, c_r;
  ActionTables tab;         // Hx, Hy in cell units per step
  double speed[kMaxA];      // F of each action
};

hipError_t launch_rollout(const RollParams &P, mdp_rollout_stats *dev_stats, hipStream_t s);

// The calling thread's current device, which must be `device`: the address of
// that device's copy of the allocation-free value-iteration scratch
// (noalloc.hip), looked up once per device.
hipError_t noalloc_scratch(int device, void **out);

}  // namespace mdpk
