// Value iteration and greedy policy on the CSR model (Sec. II-B update rule).
//
// A workgroup takes blocks of whole states (their N_a rows are contiguous) and
// computes
//     Q(s, a) = R(s, a) + (sum_k cnt_k * v_old[col_k]) / N_r      (fp64)
// with the sinks DEAD and TARGET contributing 0, then max_a through LDS. The sweep's residual max_s |v_new - v_old| is reduced on the device:
// every workgroup folds its maximum into one word with an atomic max, and the
// last workgroup to finish records the sweep, decides convergence and resets
// the accumulators for the next sweep. Later sweeps of the same call see the
// done flag and return at once, so the host enqueues sweeps without polling.
#include "mdp_internal.h"

namespace mdpk {

// Block b of the sweep as seen from this workgroup: workgroups are dealt to
// the 8 XCDs round-robin, so each XCD is given a contiguous range of state
// blocks and its L2 sees the neighbouring values those blocks gather.
__device__ inline int64_t xcd_block(int64_t j, int64_t n_blocks, int &ok)
{
  const int g = gridDim.x;
  if ((g & 7) != 0) {
    const int64_t blk = (int64_t)blockIdx.x + j * g;
    ok = blk < n_blocks;
    return blk;
  }
  const int64_t per_xcd = (n_blocks + 7) / 8;
  const int64_t l = (int64_t)(blockIdx.x >> 3) + j * (g >> 3);
  const int64_t blk = (int64_t)(blockIdx.x & 7) * per_xcd + l;
  ok = (l < per_xcd) && (blk < n_blocks);
  return blk;
}

constexpr int kChunk = 2048;  // entries staged in LDS per pass

// Q(s, a) for the states of one block into q[]: the block's entries are
// contiguous, so they are streamed with coalesced loads (col, cnt and the
// gathered value) into LDS as products, then each row's thread adds its own
// products in ascending entry order (the same order for every sweep).
__device__ inline void block_q(const VIParams &P, const double *v, int64_t s0, int nst, int64_t *rp,
                               double *prod, double *q)
{
  const int tid = threadIdx.x;
  const int nrows = nst * P.na;
  const int64_t row0 = s0 * P.na;
  // nrows + 1 pointers (up to kBlock + 1): more entries than threads
  for (int k = tid; k <= nrows; k += kBlock) rp[k] = min(max(P.row_ptr[row0 + k], (int64_t)0), P.cap);
  __syncthreads();
  const int64_t e0 = rp[0], e1 = rp[nrows];
  const int64_t my_lo = (tid < nrows) ? rp[tid] : 0, my_hi = (tid < nrows) ? rp[tid + 1] : 0;
  double acc = 0.0;
  for (int64_t c0 = e0; c0 < e1; c0 += kChunk) {
    const int n = (int)min((int64_t)kChunk, e1 - c0);
    for (int k = tid; k < n; k += kBlock) {
      const uint32_t cidx = (uint32_t)P.col[c0 + k];
      const double vv = (cidx < (uint32_t)P.ns) ? v[cidx] : 0.0;
      prod[k] = (double)P.cnt[c0 + k] * vv;
    }
    __syncthreads();
    if (tid < nrows) {
      const int64_t lo = max(my_lo, c0), hi = min(my_hi, c0 + n);
      for (int64_t k = lo; k < hi; ++k) acc += prod[k - c0];
    }
    __syncthreads();
  }
  if (tid < nrows) q[tid] = (double)P.R[row0 + tid] + acc * P.inv_nr;
  __syncthreads();
}

// One synchronous sweep over a chip-filling grid: one residual atomic per
// workgroup, the last workgroup to finish closes the sweep.
__global__ __launch_bounds__(kBlock) void k_vi_sweep(const VIParams P, const double *vin, double *vout,
                                                      int parity)
{
  __shared__ int64_t rp[kBlock + 1];
  __shared__ double prod[kChunk];
  __shared__ double q[kBlock];
  __shared__ double wmax[kBlock / 64];
  if (P.st->done) return;
  const int tid = threadIdx.x;
  double d = 0.0;
  for (int64_t j = 0;; ++j) {
    int ok;
    const int64_t blk = xcd_block(j, P.n_blocks, ok);
    if (!ok) break;
    const int64_t s0 = blk * P.states_per_wg;
    const int nst = (int)min((int64_t)P.states_per_wg, P.ns - s0);
    block_q(P, vin, s0, nst, rp, prod, q);
    if (tid < nst) {
      const double *qs = q + tid * P.na;
      double best = qs[0];
      for (int a = 1; a < P.na; ++a) best = fmax(best, qs[a]);
      const int64_t s = s0 + tid;
      vout[s] = best;
      d = fmax(d, fabs(best - vin[s]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = d;
  __syncthreads();
  if (tid == 0) {
    double m = wmax[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, wmax[w]);
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
  (void)parity;
}

__global__ void k_vi_init(VIState *st)
{
  if (threadIdx.x == 0) {
    st->res_bits = 0ull;
    st->wg_count = 0u;
    st->done = 0;
    st->sweeps = 0;
    st->status = 0;
    st->last_res = 0.0;
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
  __shared__ int64_t rp[kBlock + 1];
  __shared__ double prod[kChunk];
  __shared__ double q[kBlock];
  const int tid = threadIdx.x;
  for (int64_t j = 0;; ++j) {
    int ok;
    const int64_t blk = xcd_block(j, P.n_blocks, ok);
    if (!ok) break;
    const int64_t s0 = blk * P.states_per_wg;
    const int nst = (int)min((int64_t)P.states_per_wg, P.ns - s0);
    block_q(P, v, s0, nst, rp, prod, q);
    if (tid < nst) {
      const double *qs = q + tid * P.na;
      double best = qs[0];
      int besta = 0;
      for (int a = 1; a < P.na; ++a)
        if (qs[a] > best) {  // the lowest index wins ties
          best = qs[a];
          besta = a;
        }
      pi[s0 + tid] = besta;
    }
    __syncthreads();
  }
}

hipError_t launch_vi_init(VIState *st, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_init, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_vi_sweep(const VIParams &P, const double *vin, double *vout, int parity, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_sweep, dim3(P.n_wg), dim3(kBlock), 0, s, P, vin, vout, parity);
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

}  // namespace mdpk
