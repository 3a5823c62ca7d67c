// Value iteration and greedy policy on the CSR model (Sec. II-B update rule).
//
// A workgroup takes blocks of whole states (a state's N_a rows are
// contiguous); each thread computes two rows
//     Q(s, a) = R(s, a) + (sum_k cnt_k * v_old[col_k]) / N_r      (fp64)
// adding the terms in ascending entry order, with the sinks DEAD and TARGET
// contributing 0, then one thread per state takes max_a through LDS. The two
// rows of a thread are walked together so their loads overlap.
//
// Residual max_s |v_new - v_old|: in the single-problem sweep every workgroup
// of a chip-filling grid folds its maximum into one word and the last
// workgroup to finish closes the sweep (count, done flag, reset); later sweeps
// of the call see the done flag and return at once, so the host enqueues the
// sweeps without polling. In the batched sweep workgroups write one maximum
// per problem into a [grid][problems] matrix and a small kernel closes each
// problem's sweep (no atomics).
#include "mdp_internal.h"

namespace mdpk {

constexpr int kRowsPerBlock = 2 * kBlock;

// Q for the rows of states [s0, s0 + nst) into q[], then per state either the
// new value (returns the block's max |v_new - v_old|) or the first argmax.
template <bool POLICY>
__device__ inline double vi_block(const VIParams &P, const double *vin, double *vout, int32_t *pi, int64_t s0,
                                  int nst, double *q)
{
  const int tid = threadIdx.x;
  const int nrows = nst * P.na;
  const int64_t row0 = s0 * P.na;
  const uint32_t ns32 = (uint32_t)P.ns;
  int64_t k0 = 0, e0 = 0, k1 = 0, e1 = 0;
  if (tid < nrows) {
    k0 = P.row_ptr[row0 + tid];
    e0 = min(P.row_ptr[row0 + tid + 1], P.cap);
  }
  if (tid + kBlock < nrows) {
    k1 = P.row_ptr[row0 + tid + kBlock];
    e1 = min(P.row_ptr[row0 + tid + kBlock + 1], P.cap);
  }
  k0 = max(k0, (int64_t)0);
  k1 = max(k1, (int64_t)0);
  double a0 = 0.0, a1 = 0.0;
  while (k0 < e0 || k1 < e1) {
    if (k0 < e0) {
      const uint32_t c = (uint32_t)P.col[k0];
      const double vv = (c < ns32) ? vin[c] : 0.0;
      a0 += (double)P.cnt[k0] * vv;
      ++k0;
    }
    if (k1 < e1) {
      const uint32_t c = (uint32_t)P.col[k1];
      const double vv = (c < ns32) ? vin[c] : 0.0;
      a1 += (double)P.cnt[k1] * vv;
      ++k1;
    }
  }
  if (tid < nrows) q[tid] = (double)P.R[row0 + tid] + a0 * P.inv_nr;
  if (tid + kBlock < nrows) q[tid + kBlock] = (double)P.R[row0 + tid + kBlock] + a1 * P.inv_nr;
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
      d = fabs(best - vin[s]);
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

// One synchronous sweep over a chip-filling grid.
__global__ __launch_bounds__(kBlock) void k_vi_sweep(const VIParams P, const double *vin, double *vout)
{
  __shared__ double q[kRowsPerBlock];
  __shared__ double wmax[kBlock / 64];
  if (P.st->done) return;
  double d = 0.0;
  for (int64_t blk = blockIdx.x; blk < P.n_blocks; blk += gridDim.x) {
    const int64_t s0 = blk * P.states_per_wg;
    const int nst = (int)min((int64_t)P.states_per_wg, P.ns - s0);
    d = fmax(d, vi_block<false>(P, vin, vout, nullptr, s0, nst, q));
  }
  const double m = block_max(d, wmax);
  if (threadIdx.x == 0) {
    atomicMax(&P.st->res_bits, (unsigned long long)__double_as_longlong(m));
    __threadfence();
    const unsigned int prev = atomicAdd(&P.st->wg_count, 1u);
    if (prev == gridDim.x - 1u) {
      __threadfence();
      const unsigned long long rb = atomicAdd(&P.st->res_bits, 0ull);
      const double res = __longlong_as_double((long long)rb);
      P.st->sweeps += 1;
      P.st->last_res = res;
      if (res < P.tol) P.st->done = 1;
      P.st->res_bits = 0ull;
      P.st->wg_count = 0u;
      __threadfence();
    }
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
  __shared__ double q[kRowsPerBlock];
  for (int64_t blk = blockIdx.x; blk < P.n_blocks; blk += gridDim.x) {
    const int64_t s0 = blk * P.states_per_wg;
    const int nst = (int)min((int64_t)P.states_per_wg, P.ns - s0);
    vi_block<true>(P, v, nullptr, pi, s0, nst, q);
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

// One synchronous sweep of every problem that has not converged. A problem
// with an even sweep count reads v and writes v_alt, with an odd count the
// reverse, so problems that joined at different sweeps share the launch.
// wg_res[blockIdx][i] gets this workgroup's max residual of problem i.
__global__ __launch_bounds__(kBlock) void k_vi_sweep_batched(const BatchVIDesc *D, int n, const int64_t *block_start,
                                                              double *wg_res)
{
  __shared__ double q[kRowsPerBlock];
  __shared__ double wmax[kBlock / 64];
  __shared__ double res[kMaxBatch];
  __shared__ int64_t bstart[kMaxBatch + 1];
  const int tid = threadIdx.x;
  for (int i = tid; i <= n; i += kBlock) bstart[i] = block_start[i];
  for (int i = tid; i < n; i += kBlock) res[i] = 0.0;
  __syncthreads();
  const int64_t total = bstart[n];
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int i = batch_problem(bstart, n, g);
    const BatchVIDesc &d = D[i];
    if (d.st->done) continue;  // uniform per block
    const int64_t blk = g - bstart[i];
    const int64_t s0 = blk * d.P.states_per_wg;
    const int nst = (int)min((int64_t)d.P.states_per_wg, d.P.ns - s0);
    const bool odd = (d.st->sweeps & 1) != 0;
    const double *vin = odd ? d.v_alt : d.v;
    double *vout = odd ? d.v : d.v_alt;
    const double m = block_max(vi_block<false>(d.P, vin, vout, nullptr, s0, nst, q), wmax);
    if (tid == 0) res[i] = fmax(res[i], m);
  }
  __syncthreads();
  for (int i = tid; i < n; i += kBlock) wg_res[(int64_t)blockIdx.x * n + i] = res[i];
}

// Close the sweep of each problem (one block per problem).
__global__ __launch_bounds__(kBlock) void k_vi_close_batched(const BatchVIDesc *D, int n, int grid,
                                                              const double *wg_res, double tol)
{
  __shared__ double wmax[kBlock / 64];
  const int i = blockIdx.x;
  VIState *st = D[i].st;
  if (st->done) return;
  double m = 0.0;
  for (int w = threadIdx.x; w < grid; w += kBlock) m = fmax(m, wg_res[(int64_t)w * n + i]);
  m = block_max(m, wmax);
  if (threadIdx.x == 0) {
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
  __shared__ double q[kRowsPerBlock];
  __shared__ int64_t bstart[kMaxBatch + 1];
  for (int i = threadIdx.x; i <= n; i += kBlock) bstart[i] = block_start[i];
  __syncthreads();
  const int64_t total = bstart[n];
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int i = batch_problem(bstart, n, g);
    const BatchVIDesc &d = D[i];
    const int64_t s0 = (g - bstart[i]) * d.P.states_per_wg;
    const int nst = (int)min((int64_t)d.P.states_per_wg, d.P.ns - s0);
    vi_block<true>(d.P, d.v, nullptr, d.pi, s0, nst, q);
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_vi_init(VIState *st, int n, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_init, dim3((n + 63) / 64), dim3(64), 0, s, st, n);
  return hipGetLastError();
}

hipError_t launch_vi_sweep(const VIParams &P, const double *vin, double *vout, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_sweep, dim3(P.n_wg), dim3(kBlock), 0, s, P, vin, vout);
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
  hipLaunchKernelGGL(k_policy, dim3(P.n_wg), dim3(kBlock), 0, s, P, v, pi);
  return hipGetLastError();
}

hipError_t launch_vi_sweep_batched(const BatchVIDesc *D, int n, const int64_t *block_start, double *wg_res,
                                   int grid, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_sweep_batched, dim3(grid), dim3(kBlock), 0, s, D, n, block_start, wg_res);
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

hipError_t launch_vi_close_batched(const BatchVIDesc *D, int n, int grid, const double *wg_res, double tol,
                                   hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_close_batched, dim3(n), dim3(kBlock), 0, s, D, n, grid, wg_res, tol);
  return hipGetLastError();
}

hipError_t launch_vi_finish_batched(const BatchVIDesc *D, int n, mdp_vi_stats *out, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_finish_batched, dim3(256, n), dim3(kBlock), 0, s, D, n, out);
  return hipGetLastError();
}

hipError_t launch_policy_batched(const BatchVIDesc *D, int n, const int64_t *block_start, int grid, hipStream_t s)
{
  hipLaunchKernelGGL(k_policy_batched, dim3(grid), dim3(kBlock), 0, s, D, n, block_start);
  return hipGetLastError();
}

}  // namespace mdpk
