// Value iteration and greedy policy on the CSR model (Sec. II-B update rule).
//
// A workgroup takes a block of S cells of one decision layer t (their S * N_a
// rows are contiguous, at most 512; two rows per thread). Two rounds of
// global loads per block:
//   1. the block's entry range, its rows' entry offsets and rewards, each
//      state's old value, and the window of v_old(t + 1) that the rows can
//      reach (grid rows within the sub-grid half height of the block's rows);
//   2. the block's entries (col, cnt), coalesced, one lane per entry.
// The window goes to LDS; each lane forms cnt * v_old[col] for its entries
// (the sinks DEAD and TARGET contribute 0) and stages the products in LDS;
// then each row's thread adds its products in ascending entry order (fp64),
//     Q(s, a) = R(s, a) + (sum_k cnt_k * v_old[col_k]) / N_r,
// and one thread per state takes max_a Q (first maximum on ties). The per-row
// sum has a fixed order, so every path (single problem, batch, server) gives
// the same bits.
//
// Every transition goes from layer t to layer t + 1 or to a sink, and layer
// T - 1 reaches only sinks, so after k sweeps the layers t >= T - k hold
// their final values whatever v0 was. A layer that was already final before
// the previous sweep has its final value in both buffers; sweep k (0-based)
// therefore recomputes only layers t < T - k + 1. The skipped layers would
// reproduce their values bit for bit and add 0 to the residual, so this is
// exactly the synchronous sweep, with the same residual and sweep count.
//
// Residual max_s |v_new - v_old|: every workgroup writes its maximum (per
// problem in the batched sweep) and a small kernel closes the sweep (count,
// done flag); later sweeps see the done flag and return at once, so the host
// enqueues the sweeps without polling.
#include "mdp_internal.h"

#include <algorithm>

namespace mdpk {

constexpr int kViGridMax = 8192;

// Q of the rows of cells [c0, c0 + S) of layer t, then per state either the
// new value (returns the block's max |v_new - v_old|) or the first argmax.
template <bool POLICY>
__device__ inline double vi_block(const VIParams &P, const double *vin, double *vout, int32_t *pi, int t, int c0,
                                  double *sm, double *vwin)
{
  double *prod = sm + kViProd;
  double *q = sm + kViQ;
  const int tid = threadIdx.x;
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int nr = nst * P.na;
  const int64_t s0 = (int64_t)t * P.nc + c0;
  const int64_t row0 = s0 * P.na;
  // ---- round 1. The block's entries [eb, ee), clamped so that a malformed
  // row pointer can neither read outside col / cnt nor loop long.
  const int64_t eb = min(max(P.row_ptr[row0], (int64_t)0), P.cap);
  const int64_t ee = min(min(max(P.row_ptr[row0 + nr], eb), P.cap), eb + (int64_t)nr * P.max_row);
  const int E = (int)(ee - eb);
  int lo[2], hi[2];
  float rr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = tid + kBlock * h;
    lo[h] = hi[h] = 0;
    rr[h] = 0.0f;
    if (r < nr) {
      lo[h] = (int)(min(max(P.row_ptr[row0 + r], eb), ee) - eb);
      hi[h] = (int)(min(max(P.row_ptr[row0 + r + 1], eb), ee) - eb);
      rr[h] = P.R[row0 + r];
    }
  }
  const double vself = (!POLICY && tid < nst) ? vin[s0 + tid] : 0.0;
  int64_t wbase = 0;
  int wn = 0;
  if (P.win_rows > 0 && t + 1 < P.nt) {
    const int jw0 = max(0, c0 / P.nx - P.hy);
    const int jw1 = min(P.ny - 1, (c0 + nst - 1) / P.nx + P.hy);
    wn = (jw1 - jw0 + 1) * P.nx;  // <= win_rows * nx <= kViWinPerThread * kBlock
    wbase = (int64_t)(t + 1) * P.nc + (int64_t)jw0 * P.nx;
  }
  {
    // the window goes to LDS before the entries are loaded (their loads need
    // the block's first row pointer anyway), so its registers are free again
    double wv[kViWinPerThread];
#pragma unroll
    for (int j = 0; j < kViWinPerThread; ++j) {
      const int k = tid + kBlock * j;
      wv[j] = k < wn ? vin[wbase + k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kViWinPerThread; ++j) {
      const int k = tid + kBlock * j;
      if (k < wn) vwin[k] = wv[j];
    }
  }
  const uint32_t ns32 = (uint32_t)P.ns;
  double acc[2] = {0.0, 0.0};
  for (int base = 0; base < E; base += kViChunk) {
    const int ce = min(E - base, kViChunk);
    // ---- round 2: this chunk's entries, one lane per entry
    uint32_t cc[kViChunk / kBlock];
    uint16_t nn[kViChunk / kBlock];
#pragma unroll
    for (int j = 0; j < kViChunk / kBlock; ++j) {
      const int k = tid + kBlock * j;
      const int64_t e = eb + base + (k < ce ? k : 0);  // a valid index past the end
      cc[j] = (uint32_t)P.col[e];
      nn[j] = P.cnt[e];
    }
    __syncthreads();  // the window (first round) and the previous round's reads
#pragma unroll
    for (int j = 0; j < kViChunk / kBlock; ++j) {
      const int k = tid + kBlock * j;
      if (k < ce) {
        double vv = 0.0;
        if (cc[j] < ns32) {
          const int64_t w = (int64_t)cc[j] - wbase;
          vv = (w >= 0 && w < wn) ? vwin[w] : vin[cc[j]];
        }
        prod[k] = (double)nn[j] * vv;
      }
    }
    __syncthreads();
    // ---- each row's products in ascending order (independent LDS reads)
    const int top = base + ce;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int k = max(lo[h], base);
      const int k1 = min(hi[h], top);
      for (; k + 4 <= k1; k += 4) {
        const double x0 = prod[k - base], x1 = prod[k + 1 - base], x2 = prod[k + 2 - base], x3 = prod[k + 3 - base];
        acc[h] += x0;
        acc[h] += x1;
        acc[h] += x2;
        acc[h] += x3;
      }
      for (; k < k1; ++k) acc[h] += prod[k - base];
    }
    __syncthreads();
  }
  // q aliases the products: every row sum above has completed
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = tid + kBlock * h;
    if (r < nr) q[r] = (double)rr[h] + acc[h] * P.inv_nr;
  }
  __syncthreads();
  double d = 0.0;
  if (tid < nst) {
    const double *qs = q + tid * P.na;
    double best = qs[0];
    int besta = 0;
    for (int a = 1; a < P.na; ++a)
      if (qs[a] > best) {  // the lowest index wins ties
        best = qs[a];
        besta = a;
      }
    const int64_t s = s0 + tid;
    if (POLICY) {
      pi[s] = besta;
    } else {
      vout[s] = best;
      d = fabs(best - vself);
    }
  }
  __syncthreads();
  return d;
}

__device__ inline double block_max(double d, double *wmax)
{
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = d;
  __syncthreads();
  double m = wmax[0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, wmax[w]);
  __syncthreads();
  return m;
}

// One synchronous sweep over the blocks of layers [0, t_hi); wg_res[blockIdx]
// gets the workgroup's max |v_new - v_old|.
__global__ __launch_bounds__(kBlock) void k_vi_sweep(const VIParams P, const double *vin, double *vout, int t_hi,
                                                      double *wg_res)
{
  extern __shared__ double sm[];
  if (P.st->done) return;
  double d = 0.0;
  const int64_t nb = (int64_t)t_hi * P.blocks_per_layer;
  for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const int t = (int)(blk / P.blocks_per_layer);
    const int c0 = (int)(blk - (int64_t)t * P.blocks_per_layer) * P.states_per_wg;
    d = fmax(d, vi_block<false>(P, vin, vout, nullptr, t, c0, sm, sm + kViFixed));
  }
  const double m = block_max(d, sm + kViWmax);
  if (threadIdx.x == 0) wg_res[blockIdx.x] = m;
}

constexpr int kCloseBlock = 1024;  // threads of the sweep-closing kernel (8 partial maxima each at most)

// Close one sweep: count, last residual, done flag.
__global__ __launch_bounds__(kCloseBlock) void k_vi_close(const VIParams P, const double *wg_res, int grid)
{
  __shared__ double wmax[kCloseBlock / 64];
  VIState *st = P.st;
  if (st->done) return;
  double m = 0.0;
  for (int w = threadIdx.x; w < grid; w += kCloseBlock) m = fmax(m, wg_res[w]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCloseBlock / 64; ++w) m = fmax(m, wmax[w]);
    st->sweeps += 1;
    st->last_res = m;
    if (m < P.tol) st->done = 1;
  }
}

__global__ void k_vi_init(VIState *st, int n)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    st[i].res_bits = 0ull;
    st[i].wg_count = 0u;
    st[i].done = 0;
    st[i].sweeps = 0;
    st[i].status = 0;
    st[i].last_res = 0.0;
  }
}

// After the sweeps: the result sits in v after an even number of sweeps and in
// v_alt after an odd number; bring it back into v and publish the stats.
__global__ __launch_bounds__(kBlock) void k_vi_finish(const VIParams P, double *v, const double *v_alt,
                                                       mdp_vi_stats *out)
{
  const int sweeps = P.st->sweeps;
  if (sweeps & 1) {
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < P.ns; s += (int64_t)gridDim.x * kBlock)
      v[s] = v_alt[s];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out->sweeps = sweeps;
    out->residual = P.st->last_res;
    out->status = P.st->done ? MDP_OK : MDP_E_NOT_CONVERGED;
  }
}

__global__ __launch_bounds__(kBlock) void k_policy(const VIParams P, const double *v, int32_t *pi)
{
  extern __shared__ double sm[];
  for (int64_t blk = blockIdx.x; blk < P.n_blocks; blk += gridDim.x) {
    const int t = (int)(blk / P.blocks_per_layer);
    const int c0 = (int)(blk - (int64_t)t * P.blocks_per_layer) * P.states_per_wg;
    vi_block<true>(P, v, nullptr, pi, t, c0, sm, sm + kViFixed);
  }
}

// ------------------------------------------------------------------ batches
// Problem owning global block g: block_start is ascending with n + 1 entries.
__device__ inline int batch_problem(const int64_t *block_start, int n, int64_t g)
{
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (block_start[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One synchronous sweep of every problem that has not converged. block_start
// lists, per problem, the blocks of the layers this sweep recomputes (layers
// t < nt - k + 1 after k sweeps, computed by the host). A problem with an even
// sweep count reads v and writes v_alt, with an odd count the reverse, so
// problems that joined at different sweeps share the launch. Sweep counts and
// done flags are read once per workgroup. wg_res[blockIdx][i] gets this
// workgroup's max residual of problem i.
__global__ __launch_bounds__(kBlock) void k_vi_sweep_batched(const BatchVIDesc *D, int n, const int64_t *block_start,
                                                              double *wg_res)
{
  extern __shared__ double sm[];
  double *res = sm + kViFixed;
  int64_t *bstart = reinterpret_cast<int64_t *>(sm + kViFixed + n);
  int2 *stc = reinterpret_cast<int2 *>(sm + kViFixed + 2 * n + 1);  // (sweeps, done) per problem
  double *vwin = sm + kViFixed + 3 * n + 1;
  const int tid = threadIdx.x;
  for (int i = tid; i <= n; i += kBlock) bstart[i] = block_start[i];
  for (int i = tid; i < n; i += kBlock) {
    res[i] = 0.0;
    const VIState *st = D[i].st;
    stc[i] = make_int2(st->sweeps, st->done);
  }
  __syncthreads();
  // a contiguous range of blocks per workgroup, so consecutive blocks share a
  // problem; the problem index is wave-uniform, so descriptor loads are scalar
  const int64_t total = bstart[n];
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t g_end = min(total, (int64_t)(blockIdx.x + 1) * per);
  for (int64_t g = (int64_t)blockIdx.x * per; g < g_end; ++g) {
    const int i = __builtin_amdgcn_readfirstlane(batch_problem(bstart, n, g));
    const int2 sd = stc[i];
    if (sd.y) continue;  // converged (uniform per block)
    const BatchVIDesc d = load_const(D + i);
    const VIParams &P = d.P;
    const int64_t blk = g - bstart[i];
    const int t = (int)(blk / P.blocks_per_layer);
    if (t >= vi_active_layers(P.nt, sd.x)) continue;
    const int c0 = (int)(blk - (int64_t)t * P.blocks_per_layer) * P.states_per_wg;
    const bool odd = (sd.x & 1) != 0;
    const double *vin = odd ? d.v_alt : d.v;
    double *vout = odd ? d.v : d.v_alt;
    const double m = block_max(vi_block<false>(P, vin, vout, nullptr, t, c0, sm, vwin), sm + kViWmax);
    if (tid == 0) res[i] = fmax(res[i], m);
  }
  __syncthreads();
  for (int i = tid; i < n; i += kBlock) wg_res[(int64_t)blockIdx.x * n + i] = res[i];
}

// Close the sweep of each problem (one block per problem).
__global__ __launch_bounds__(kCloseBlock) void k_vi_close_batched(const BatchVIDesc *D, int n, int grid,
                                                                   const double *wg_res, double tol)
{
  __shared__ double wmax[kCloseBlock / 64];
  const int i = blockIdx.x;
  VIState *st = D[i].st;
  if (st->done) return;
  double m = 0.0;
  for (int w = threadIdx.x; w < grid; w += kCloseBlock) m = fmax(m, wg_res[(int64_t)w * n + i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCloseBlock / 64; ++w) m = fmax(m, wmax[w]);
    st->sweeps += 1;
    st->last_res = m;
    if (m < tol) st->done = 1;
  }
}

// Results back into v (odd sweep counts) and the stats of each problem.
__global__ __launch_bounds__(kBlock) void k_vi_finish_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out)
{
  const int i = blockIdx.y;
  const BatchVIDesc &d = D[i];
  const int sweeps = d.st->sweeps;
  if (sweeps & 1) {
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < d.P.ns; s += (int64_t)gridDim.x * kBlock)
      d.v[s] = d.v_alt[s];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[i].sweeps = sweeps;
    out[i].residual = d.st->last_res;
    out[i].status = d.st->done ? MDP_OK : MDP_E_NOT_CONVERGED;
  }
}

// Cold start of problems joining a running batch: v = 0 and a fresh sweep
// state (grid.y = problem).
__global__ __launch_bounds__(kBlock) void k_vi_reset_batched(const BatchVIDesc *D)
{
  const BatchVIDesc &d = D[blockIdx.y];
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < d.P.ns; s += (int64_t)gridDim.x * kBlock)
    d.v[s] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    VIState *st = d.st;
    st->res_bits = 0ull;
    st->wg_count = 0u;
    st->done = 0;
    st->sweeps = 0;
    st->status = 0;
    st->last_res = 0.0;
  }
}

// Sweep count, convergence and last residual of every problem, without
// touching the values (one thread per problem).
__global__ void k_vi_status_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const VIState *st = D[i].st;
    out[i].sweeps = st->sweeps;
    out[i].status = st->done ? MDP_OK : MDP_E_NOT_CONVERGED;
    out[i].residual = st->last_res;
  }
}

__global__ __launch_bounds__(kBlock) void k_policy_batched(const BatchVIDesc *D, int n, const int64_t *block_start)
{
  extern __shared__ double sm[];
  int64_t *bstart = reinterpret_cast<int64_t *>(sm + kViFixed + n);
  double *vwin = sm + kViFixed + 3 * n + 1;
  for (int i = threadIdx.x; i <= n; i += kBlock) bstart[i] = block_start[i];
  __syncthreads();
  const int64_t total = bstart[n];
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t g_end = min(total, (int64_t)(blockIdx.x + 1) * per);
  for (int64_t g = (int64_t)blockIdx.x * per; g < g_end; ++g) {
    const int i = __builtin_amdgcn_readfirstlane(batch_problem(bstart, n, g));
    const BatchVIDesc d = load_const(D + i);
    const VIParams &P = d.P;
    const int64_t blk = g - bstart[i];
    const int t = (int)(blk / P.blocks_per_layer);
    const int c0 = (int)(blk - (int64_t)t * P.blocks_per_layer) * P.states_per_wg;
    vi_block<true>(P, d.v, nullptr, d.pi, t, c0, sm, vwin);
  }
}

// ------------------------------------------------------------------ launchers
// Raise a kernel's dynamic-LDS limit to whatever its static LDS leaves free.
static hipError_t allow_lds(const void *kern, bool &done)
{
  if (done) return hipSuccess;
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, kern);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - fa.sharedSizeBytes));
  if (e == hipSuccess) done = true;
  return e;
}

static size_t single_lds(const VIParams &P) { return (size_t)kViFixed * 8 + (size_t)P.win_rows * P.nx * 8; }

static size_t batch_lds(int n, size_t win_bytes) { return ((size_t)kViFixed + 3 * (size_t)n + 2) * 8 + win_bytes; }

hipError_t launch_vi_init(VIState *st, int n, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_init, dim3((n + 63) / 64), dim3(64), 0, s, st, n);
  return hipGetLastError();
}

hipError_t launch_vi_sweep(const VIParams &P, const double *vin, double *vout, int t_hi, double *wg_res,
                           hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_vi_sweep, attr);
  if (e != hipSuccess) return e;
  const int64_t nb = (int64_t)t_hi * P.blocks_per_layer;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nb, std::min(P.n_wg, kViGridMax)));
  hipLaunchKernelGGL(k_vi_sweep, dim3(grid), dim3(kBlock), single_lds(P), s, P, vin, vout, t_hi, wg_res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_vi_close, dim3(1), dim3(kCloseBlock), 0, s, P, (const double *)wg_res, grid);
  return hipGetLastError();
}

hipError_t launch_vi_finish(const VIParams &P, double *v, const double *v_alt, mdp_vi_stats *dev_stats,
                            hipStream_t s)
{
  const int64_t nb = (P.ns + kBlock - 1) / kBlock;
  const int grid = (int)(nb < 4096 ? nb : 4096);
  hipLaunchKernelGGL(k_vi_finish, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, s, P, v, v_alt, dev_stats);
  return hipGetLastError();
}

hipError_t launch_policy(const VIParams &P, const double *v, int32_t *pi, hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_policy, attr);
  if (e != hipSuccess) return e;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(P.n_blocks, kViGridMax));
  hipLaunchKernelGGL(k_policy, dim3(grid), dim3(kBlock), single_lds(P), s, P, v, pi);
  return hipGetLastError();
}

hipError_t launch_vi_sweep_batched(const BatchVIDesc *D, int n, const int64_t *block_start, double *wg_res,
                                   int grid, size_t win_bytes, hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_vi_sweep_batched, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vi_sweep_batched, dim3(grid), dim3(kBlock), batch_lds(n, win_bytes), s, D, n, block_start,
                     wg_res);
  return hipGetLastError();
}

hipError_t launch_vi_close_batched(const BatchVIDesc *D, int n, int grid, const double *wg_res, double tol,
                                   hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_close_batched, dim3(n), dim3(kCloseBlock), 0, s, D, n, grid, wg_res, tol);
  return hipGetLastError();
}

hipError_t launch_vi_finish_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_finish_batched, dim3(256, n), dim3(kBlock), 0, s, D, n, out);
  return hipGetLastError();
}

hipError_t launch_vi_reset_batched(const BatchVIDesc *D, int n, hipStream_t s)
{
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_vi_reset_batched, dim3(64, n), dim3(kBlock), 0, s, D);
  return hipGetLastError();
}

hipError_t launch_vi_status_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out, hipStream_t s)
{
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_vi_status_batched, dim3((n + 63) / 64), dim3(64), 0, s, D, n, out);
  return hipGetLastError();
}

hipError_t launch_policy_batched(const BatchVIDesc *D, int n, const int64_t *block_start, int grid,
                                 size_t win_bytes, hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_policy_batched, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_policy_batched, dim3(grid), dim3(kBlock), batch_lds(n, win_bytes), s, D, n, block_start);
  return hipGetLastError();
}

}  // namespace mdpk
