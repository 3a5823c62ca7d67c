// Value iteration and greedy policy on the CSR model (Sec. II-B update rule).
//
// A workgroup takes a block of S cells of one decision layer t (their S * N_a
// rows are contiguous, at most 512; two rows per thread). The block's entry
// range (its first and one-past-last row pointer) is read with scalar loads
// while the previous block of the workgroup is processed, so one round of
// loads per block suffices, all issued together and branch-free:
//   - its rows' entry offsets and rewards and each state's old value;
//   - the window of v_old(t + 1) that the rows can reach (grid rows within
//     the sub-grid half height of the block's rows), copied by the memory
//     unit straight into LDS (global_load_lds), which costs no registers;
//   - its entries (col, cnt), coalesced, one lane per entry, up to 2048.
// Each lane forms cnt * v_old[col] for its entries (a window read in LDS; the
// sinks DEAD and TARGET contribute 0; a state outside the window, possible
// only when the window is off, is read from HBM) and stages the products in
// LDS; then each row's thread adds its products in ascending entry order
// (fp64),
//     Q(s, a) = R(s, a) + (sum_k cnt_k * v_old[col_k]) / N_r,
// writes Q back to LDS at an odd stride per state, and one thread per state
// takes max_a Q (first maximum on ties) without bank conflicts. The per-row
// sum has a fixed order, so every path (single problem, batch, server, several
// missions at once) gives the same bits.
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

constexpr int kViGridMax = 8192;  // a multiple of kXcds
constexpr int kXcds = 8;          // compute chiplets (XCDs) of an MI355X

typedef __attribute__((address_space(1))) void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;

// s_waitcnt vmcnt(0): every vector memory load of this wave has completed,
// including the copies that write LDS directly.
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// First maximum of qs[0 .. na): the largest value and the lowest index
// attaining it. Reads go out in groups of 8 independent LDS loads (indices
// past na repeat qs[na - 1], which a strict comparison never takes).
__device__ inline double first_max(const double *qs, int na, int &besta)
{
  double best = qs[0];
  besta = 0;
  for (int a0 = 0; a0 < na; a0 += 8) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = qs[min(a0 + j, na - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (x[j] > best) {  // the lowest index wins ties
        best = x[j];
        besta = a0 + j;
      }
  }
  return best;
}

// Entry range [rb, re) of the block of cells [c0, c0 + S) of layer t, as
// stored (unclamped): the first and the one-past-last row pointer.
struct RowSpan {
  int64_t rb, re;
};

__device__ inline RowSpan block_span(const VIParams &P, int t, int c0)
{
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int64_t row0 = ((int64_t)t * P.nc + c0) * P.na;
  // uniform: scalar loads through the constant address space
  return RowSpan{load_const(P.row_ptr + row0), load_const(P.row_ptr + row0 + (int64_t)nst * P.na)};
}

// Q of the rows of cells [c0, c0 + S) of layer t, then per state either the
// new value (returns the block's max |v_new - v_old|) or the first argmax.
// `span` is the block's entry range (block_span), known before the block
// starts, so its entries are loaded in the same round as its rows' data.
template <bool POLICY>
__device__ inline double vi_block(const VIParams &P, const double *vin, double *vout, int32_t *pi, int t, int c0,
                                  RowSpan span, double *sm, double *vwin)
{
  double *prod = sm + kViProd;
  double *q = sm + kViQ;
  const int tid = threadIdx.x;
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int nr = nst * P.na;
  const int64_t s0 = (int64_t)t * P.nc + c0;
  const int64_t row0 = s0 * P.na;
  // The block's entries [eb, ee), clamped so that a malformed row pointer can
  // neither read outside col / cnt nor loop long.
  const int64_t eb = min(max(span.rb, (int64_t)0), P.cap);
  const int64_t ee = min(min(max(span.re, eb), P.cap), eb + (int64_t)nr * P.max_row);
  const int E = (int)(ee - eb);
  // ---- one round of loads: rows' entry offsets and rewards, own values, the
  // window of v_old(t + 1), and the first chunk of entries
  // (branch-free: indices are clamped to valid rows and the results masked
  // afterwards, so every load of the round is in flight at once)
  int64_t rlo[2], rhi[2];
  float rr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = min(tid + kBlock * h, nr);
    rlo[h] = P.row_ptr[row0 + r];
    rhi[h] = P.row_ptr[row0 + r + (r < nr)];
    rr[h] = P.R[row0 + min(r, nr - 1)];
  }
  const double vself = POLICY ? 0.0 : vin[s0 + min(tid, nst - 1)];
  int64_t wbase = 0;
  int wn = 0;
  if (P.win_rows > 0 && t + 1 < P.nt) {
    const int jw0 = max(0, c0 / P.nx - P.hy);
    const int jw1 = min(P.ny - 1, (c0 + nst - 1) / P.nx + P.hy);
    wn = (jw1 - jw0 + 1) * P.nx;  // <= win_rows * nx <= kViWinPerThread * kBlock
    wbase = (int64_t)(t + 1) * P.nc + (int64_t)jw0 * P.nx;
  }
  // the window goes straight to LDS (no registers): dword copies, one wave
  // row of 64 dwords per instruction
  {
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const char *src = reinterpret_cast<const char *>(vin + wbase);
    char *dst = reinterpret_cast<char *>(vwin);
    for (int j = wave * 64; j < 2 * wn; j += kBlock) {
      if (j + lane < 2 * wn)
        __builtin_amdgcn_global_load_lds((gptr_t)(src + 4 * (size_t)(j + lane)), (lptr_t)(dst + 4 * (size_t)j), 4, 0,
                                         0);
    }
  }
  uint32_t cc[kViChunk / kBlock];
  uint16_t nn[kViChunk / kBlock];
  // a model without entries (cap 0) reads its row pointers instead: every
  // index below is valid, so the loads need no branch
  const uint32_t *colp = P.cap > 0 ? reinterpret_cast<const uint32_t *>(P.col)
                                   : reinterpret_cast<const uint32_t *>(P.row_ptr);
  const uint16_t *cntp = P.cap > 0 ? P.cnt : reinterpret_cast<const uint16_t *>(P.row_ptr);
  const int64_t elast = max(P.cap - 1, (int64_t)0);
  auto load_chunk = [&](int base) {
    const int ce = min(E - base, kViChunk);
#pragma unroll
    for (int j = 0; j < kViChunk / kBlock; ++j) {
      const int k = tid + kBlock * j;
      const int64_t e = min(eb + base + (k < ce ? k : 0), elast);
      cc[j] = colp[e];
      nn[j] = cntp[e];
    }
  };
  load_chunk(0);  // unconditional, so that no load waits for another
  int lo[2], hi[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    lo[h] = (int)(min(max(rlo[h], eb), ee) - eb);
    hi[h] = (int)(min(max(rhi[h], eb), ee) - eb);
  }
  const uint32_t ns32 = (uint32_t)P.ns;
  const uint32_t wbase32 = (uint32_t)wbase;
  double acc[2] = {0.0, 0.0};
  for (int base = 0; base < E; base += kViChunk) {
    const int ce = min(E - base, kViChunk);
    if (base > 0) load_chunk(base);  // further chunks: one more round each
    wait_vm();        // this wave's window copies have landed in LDS
    __syncthreads();  // every wave's, and the previous round's reads are done
    // v_old of every entry's successor: one LDS read per entry, branch-free
    // (index 0 outside the window, sinks give 0), then global reads for the
    // rare states outside the window. Slots past the round's entries hold a
    // valid entry; their products land past the rows' ranges, never summed.
    constexpr int kHalf = kViChunk / kBlock / 2;  // in two halves, to bound registers
#pragma unroll
    for (int j0 = 0; j0 < kViChunk / kBlock; j0 += kHalf) {
      double vv[kHalf];
      uint32_t outside = 0;
#pragma unroll
      for (int j = 0; j < kHalf; ++j) {
        // 32-bit: states and window bases are below 2^31; sinks are never inside
        const uint32_t w = cc[j0 + j] - wbase32;
        const bool inw = w < (uint32_t)wn;
        const double x = vwin[inw ? w : 0u];
        vv[j] = inw ? x : 0.0;
        outside |= (uint32_t)(!inw && cc[j0 + j] < ns32) << j;
      }
      if (outside) {
#pragma unroll
        for (int j = 0; j < kHalf; ++j)
          if (outside >> j & 1) vv[j] = vin[cc[j0 + j]];
      }
#pragma unroll
      for (int j = 0; j < kHalf; ++j) prod[tid + kBlock * (j0 + j)] = (double)nn[j0 + j] * vv[j];
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
  // q aliases the products: every row sum above has completed. A state's Q
  // values sit at an odd stride (N_a, or N_a + 1 when N_a is even), so the
  // lanes reading one action each of consecutive states hit distinct banks.
  const int qstride = P.na | 1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = tid + kBlock * h;
    if (r < nr) q[r + (qstride - P.na) * (r / P.na)] = (double)rr[h] + acc[h] * P.inv_nr;
  }
  __syncthreads();
  double d = 0.0;
  if (tid < nst) {
    int besta = 0;
    const double best = first_max(q + tid * qstride, P.na, besta);
    const int64_t s = s0 + tid;
    if (POLICY) {
      pi[s] = besta;
    } else {
      vout[s] = best;
      d = fabs(best - vself);
    }
  }
  wait_vm();  // no copy into LDS outlives the block (a block without entries never waited)
  __syncthreads();
  return d;
}

// The blocks of layers [0, t_hi) a workgroup takes. Workgroups are dispatched
// round-robin over the kXcds chiplets (workgroup w on chiplet w % kXcds), each
// with its own L2; chiplet x takes the contiguous range x of kXcds equal
// ranges of the layer-major block order, so a layer's window of v_old(t + 1)
// is fetched from HBM by (about) one chiplet instead of all of them. Within a
// range the chiplet's workgroups stride by their count; each block's entry
// range is loaded while the previous block is processed. Needs gridDim.x to
// be a multiple of kXcds.
template <typename F>
__device__ inline void for_blocks(const VIParams &P, int t_hi, F &&body)
{
  const int bpl = P.blocks_per_layer;
  const int t_lo = min(P.t_lo, t_hi);      // layers [t_lo, t_hi)
  const int b0 = t_lo * bpl;
  const int nb = (t_hi - t_lo) * bpl;      // < 2^31: the state count fits 32 bits
  const int x = (int)blockIdx.x % kXcds, nslot = (int)gridDim.x / kXcds;
  const int b_end = b0 + (int)((int64_t)nb * (x + 1) / kXcds);
  int b = b0 + (int)((int64_t)nb * x / kXcds) + (int)blockIdx.x / kXcds;
  if (b >= b_end) return;
  const int gq = nslot / bpl, gr = nslot % bpl;
  int t = b / bpl, c = b - t * bpl;
  RowSpan span = block_span(P, t, c * P.states_per_wg);
  for (; b < b_end; b += nslot) {
    int tn = t + gq, cn = c + gr;
    if (cn >= bpl) {
      cn -= bpl;
      ++tn;
    }
    RowSpan nxt{0, 0};
    if ((int64_t)b + nslot < b_end) nxt = block_span(P, tn, cn * P.states_per_wg);
    body(t, c * P.states_per_wg, span);
    t = tn;
    c = cn;
    span = nxt;
  }
}

// Workgroups of a sweep or policy launch over nb blocks: a multiple of kXcds.
inline int vi_grid(int64_t nb, int cap)
{
  const int64_t g = std::min<int64_t>(std::max<int64_t>(nb, 1), cap);
  return (int)((g + kXcds - 1) / kXcds * kXcds);
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
  for_blocks(P, t_hi, [&](int t, int c0, RowSpan span) {
    d = fmax(d, vi_block<false>(P, vin, vout, nullptr, t, c0, span, sm, sm + kViFixed));
  });
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
// v_alt after an odd number; bring it back into v (the states of the layers the
// sweeps recomputed, t >= P.t_lo) and publish the stats.
__global__ __launch_bounds__(kBlock) void k_vi_finish(const VIParams P, double *v, const double *v_alt,
                                                       mdp_vi_stats *out)
{
  const int sweeps = P.st->sweeps;
  if (sweeps & 1) {
    const int64_t s0 = (int64_t)P.t_lo * P.nc;
    for (int64_t s = s0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; s < P.ns; s += (int64_t)gridDim.x * kBlock)
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
  for_blocks(P, P.nt, [&](int t, int c0, RowSpan span) {
    vi_block<true>(P, v, nullptr, pi, t, c0, span, sm, sm + kViFixed);
  });
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
    const double m =
        block_max(vi_block<false>(P, vin, vout, nullptr, t, c0, block_span(P, t, c0), sm, vwin), sm + kViWmax);
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
    vi_block<true>(P, d.v, nullptr, d.pi, t, c0, block_span(P, t, c0), sm, vwin);
  }
}

// ------------------------------------------------------------------ missions
// Entries per round of the fused sweep: at most kViChunk, at least 1.5 rows
// per thread (the room Q takes at an odd stride). Small rounds keep registers
// and LDS (products, one window per mission) low enough for six or seven
// workgroups per CU; the next round's loads overlap the last mission's sums.
constexpr int mvi_chunk(int M) { return M == 3 ? 768 : 1024; }
constexpr int mvi_waves(int M) { return M == 3 ? 7 : (M == 2 ? 6 : 7); }  // per SIMD, the occupancy aimed at
static_assert(mvi_chunk(3) >= kViRows + kViRows / 2 && mvi_chunk(3) <= kViChunk, "fused chunk size");
// Several missions of one model in one sweep (models without packed entries;
// packed ones take the row sweep below). A block's row offsets and entries
// are read from HBM once, into registers; the missions that have not
// converged then take turns over them, each with its own window of v_old(t + 1)
// (copied to LDS at the start), products, row sums (ascending, as in the single
// sweep), Q at the same odd stride and first argmax. Every mission keeps its
// own rewards, residual, sweep count (buffer parity) and done flag, so its
// iterates are those of the single-mission sweep bit for bit.
template <int M>
__device__ inline void vi_block_missions(const MultiVI &V, int live, int odd, int t, int c0, RowSpan span,
                                         double *sm, int win, double *dres)
{
  constexpr int CHM = mvi_chunk(M);
  const VIParams &P = V.d[0].P;
  double *prod = sm;  // products, then Q, of one mission at a time
  const int tid = threadIdx.x;
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int nr = nst * P.na;
  const int64_t s0 = (int64_t)t * P.nc + c0;
  const int64_t row0 = s0 * P.na;
  // this sweep's input and output buffers of mission m (uniform)
  auto vin = [&](int m) -> const double * { return (odd >> m & 1) ? V.d[m].v_alt : V.d[m].v; };
  auto vout = [&](int m) -> double * { return (odd >> m & 1) ? V.d[m].v : V.d[m].v_alt; };
  const int64_t eb = min(max(span.rb, (int64_t)0), P.cap);
  const int64_t ee = min(min(max(span.re, eb), P.cap), eb + (int64_t)nr * P.max_row);
  const int E = (int)(ee - eb);
  // ---- one round of loads, branch-free as in the single sweep
  int64_t rlo[2], rhi[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = min(tid + kBlock * h, nr);
    rlo[h] = P.row_ptr[row0 + r];
    rhi[h] = P.row_ptr[row0 + r + (r < nr)];
  }
  float rr[M][2];
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) rr[m][h] = V.d[m].P.R[row0 + min(tid + kBlock * h, nr - 1)];
  }
  // the block's window of v(t + 1): whole grid rows
  int64_t wbase = 0;
  int wn = 0;
  if (P.win_rows > 0 && t + 1 < P.nt) {
    const BlockWin bw = block_window(P, t, c0, nst, false);
    wbase = bw.base;
    wn = bw.rows * bw.cols;  // <= win_rows * nx = win
  }
  // each mission's window and own old values go straight to LDS
  double *vwin0 = sm + CHM + 8;       // after the products and the block_max slots
  double *vself0 = vwin0 + M * win;  // [M][S]
  {
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!(live >> m & 1)) continue;  // uniform
      const char *src = reinterpret_cast<const char *>(vin(m) + wbase);
      char *dst = reinterpret_cast<char *>(vwin0 + m * win);
      for (int j = wave * 64; j < 2 * wn; j += kBlock) {  // whole rows: one contiguous range
        if (j + lane < 2 * wn)
          __builtin_amdgcn_global_load_lds((gptr_t)(src + 4 * (size_t)(j + lane)), (lptr_t)(dst + 4 * (size_t)j), 4,
                                           0, 0);
      }
      src = reinterpret_cast<const char *>(vin(m) + s0);
      dst = reinterpret_cast<char *>(vself0 + m * P.states_per_wg);
      for (int j = wave * 64; j < 2 * nst; j += kBlock) {
        if (j + lane < 2 * nst)
          __builtin_amdgcn_global_load_lds((gptr_t)(src + 4 * (size_t)(j + lane)), (lptr_t)(dst + 4 * (size_t)j), 4,
                                           0, 0);
      }
    }
  }
  uint32_t cc[CHM / kBlock];
  uint16_t nn[CHM / kBlock];
  const uint32_t *colp =
      P.cap > 0 ? reinterpret_cast<const uint32_t *>(P.col) : reinterpret_cast<const uint32_t *>(P.row_ptr);
  const uint16_t *cntp = P.cap > 0 ? P.cnt : reinterpret_cast<const uint16_t *>(P.row_ptr);
  const int64_t elast = max(P.cap - 1, (int64_t)0);
  auto load_chunk = [&](int base) {
    const int ce = min(E - base, CHM);
#pragma unroll
    for (int j = 0; j < CHM / kBlock; ++j) {
      const int k = tid + kBlock * j;
      const int64_t e = min(eb + base + (k < ce ? k : 0), elast);
      cc[j] = colp[e];
      nn[j] = cntp[e];
    }
  };
  load_chunk(0);
  int lo[2], hi[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    lo[h] = (int)(min(max(rlo[h], eb), ee) - eb);
    hi[h] = (int)(min(max(rhi[h], eb), ee) - eb);
  }
  const uint32_t ns32 = (uint32_t)P.ns;
  const uint32_t wbase32 = (uint32_t)wbase;
  double acc[M][2];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m][0] = acc[m][1] = 0.0;
  // With the last mission iterating, the next chunk's loads are issued once
  // its products are formed (the chunk's entries are used up), overlapping
  // its sums; otherwise at the top of the next round.
  const bool early = (live >> (M - 1) & 1) != 0;
  for (int base = 0; base < E; base += CHM) {
    const int ce = min(E - base, CHM);
    const int top = base + ce;
    if (base > 0 && !early) load_chunk(base);
    wait_vm();  // this chunk's entries, and (first round) this wave's copies
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!(live >> m & 1)) continue;
      const double *vw = vwin0 + m * win;
      __syncthreads();  // every wave's copies; the previous readers of prod
      constexpr int kHalf = CHM / kBlock / 2;
#pragma unroll
      for (int j0 = 0; j0 < CHM / kBlock; j0 += kHalf) {
        double vv[kHalf];
        uint32_t outside = 0;
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          // 32-bit: states and window bases are below 2^31; sinks are never inside
          const uint32_t w = cc[j0 + j] - wbase32;
          const bool inw = w < (uint32_t)wn;
          const double x = vw[inw ? w : 0u];
          vv[j] = inw ? x : 0.0;
          outside |= (uint32_t)(!inw && cc[j0 + j] < ns32) << j;
        }
        if (outside) {
          const double *src = vin(m);
#pragma unroll
          for (int j = 0; j < kHalf; ++j)
            if (outside >> j & 1) vv[j] = src[cc[j0 + j]];
        }
        // slots past the round's entries hold a valid entry; their products
        // land past the rows' ranges and are never summed
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          prod[tid + kBlock * (j0 + j)] = (double)nn[j0 + j] * vv[j];
        }
      }
      if (m == M - 1 && top < E) load_chunk(top);  // (mission M - 1 is live: early)
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int k = max(lo[h], base);
        const int k1 = min(hi[h], top);
        for (; k + 4 <= k1; k += 4) {
          const double x0 = prod[k - base], x1 = prod[k + 1 - base], x2 = prod[k + 2 - base],
                       x3 = prod[k + 3 - base];
          acc[m][h] += x0;
          acc[m][h] += x1;
          acc[m][h] += x2;
          acc[m][h] += x3;
        }
        for (; k < k1; ++k) acc[m][h] += prod[k - base];
      }
    }
  }
  const int qstride = P.na | 1;
  wait_vm();  // the own-value copies (a block without entries has not waited yet)
#pragma unroll
  for (int m = 0; m < M; ++m) {
    dres[m] = 0.0;
    if (!(live >> m & 1)) continue;
    __syncthreads();  // the previous readers of prod; every wave's copies
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = tid + kBlock * h;
      if (r < nr) prod[r + (qstride - P.na) * (r / P.na)] = (double)rr[m][h] + acc[m][h] * V.d[m].P.inv_nr;
    }
    __syncthreads();
    if (tid < nst) {
      int besta;
      const double best = first_max(prod + tid * qstride, P.na, besta);
      vout(m)[s0 + tid] = best;
      dres[m] = fabs(best - vself0[m * P.states_per_wg + tid]);
    }
  }
  wait_vm();  // no copy into LDS outlives the block
  __syncthreads();
}

template <int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(mvi_waves(M), 8))) void k_vi_sweep_missions(
    const MultiVI V, int t_hi, int win, double *wg_res)
{
  extern __shared__ double sm[];
  int live = 0, odd = 0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const VIState *st = V.d[m].st;
    live |= (st->done == 0) << m;
    odd |= (st->sweeps & 1) << m;
  }
  live = __builtin_amdgcn_readfirstlane(live);
  odd = __builtin_amdgcn_readfirstlane(odd);
  if (!live) return;  // every mission has converged
  double d[M], dres[M];
#pragma unroll
  for (int m = 0; m < M; ++m) d[m] = 0.0;
  for_blocks(V.d[0].P, t_hi, [&](int t, int c0, RowSpan span) {
    vi_block_missions<M>(V, live, odd, t, c0, span, sm, win, dres);
#pragma unroll
    for (int m = 0; m < M; ++m) d[m] = fmax(d[m], dres[m]);
  });
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double mx = block_max(d[m], sm + mvi_chunk(M));
    if (threadIdx.x == 0) wg_res[(int64_t)blockIdx.x * M + m] = mx;
  }
}

// ------------------------------------------------------------------ packed rows
// The fused sweep over a packed model, one thread per row: the thread loads
// its rows' packed entries itself (the row offsets of a block are read while
// the previous block is swept), so a block waits on memory once: its entries,
// rewards, window and own-value copies are all in flight together. Each row
// sums count x v(window index) in ascending entry order from 0, as the staged
// sweep does, so the values are those of the single-mission sweep bit for bit.
constexpr int kRowUnroll = 8;      // entries of a row loaded at once; longer rows load the rest in passes
constexpr int kRowQ = kViRows + kViRows / 2;  // Q of the block's rows at the odd stride
constexpr uint32_t kNoOff = 0xFFFFu;          // no offset: a row past the block (as a start: none; as an end: E)

// Offsets of this thread's two rows (tid, tid + kBlock) of the block of cells
// [c0, c0 + nst) of layer t: start | end << 16, kNoOff past the block.
__device__ inline void load_row_offsets(const VIParams &P, int t, int c0, uint32_t (&orow)[2])
{
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int nr = nst * P.na;
  const int64_t row0 = ((int64_t)t * P.nc + c0) * P.na;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = threadIdx.x + kBlock * h;
    const uint32_t o0 = r < nr ? (uint32_t)P.roff[row0 + r] : kNoOff;
    const uint32_t o1 = r + 1 < nr ? (uint32_t)P.roff[row0 + r + 1] : kNoOff;
    orow[h] = o0 | o1 << 16;
  }
}

template <int M, typename Prefetch>
__device__ inline void vi_block_rows(const MultiVI &V, int live, int odd, int t, int c0, RowSpan span,
                                     const uint32_t (&orow)[2], Prefetch &&prefetch, double *sm, int win,
                                     double *dres)
{
  const VIParams &P = V.d[0].P;
  double *qbuf = sm;  // Q of one mission at a time
  const int tid = threadIdx.x;
  const int nst = min(P.states_per_wg, P.nc - c0);
  const int nr = nst * P.na;
  const int64_t s0 = (int64_t)t * P.nc + c0;
  const int64_t row0 = s0 * P.na;
  auto vin = [&](int m) -> const double * { return (odd >> m & 1) ? V.d[m].v_alt : V.d[m].v; };
  auto vout = [&](int m) -> double * { return (odd >> m & 1) ? V.d[m].v : V.d[m].v_alt; };
  const int64_t eb = min(max(span.rb, (int64_t)0), P.cap);
  const int64_t ee = min(min(max(span.re, eb), P.cap), eb + (int64_t)nr * P.max_row);
  const int E = (int)(ee - eb);
  // The block's entries [eb, ee): a row's entry j < len lies below ee <= cap.
  const uint32_t *entb = P.ent + eb;
  // ---- this thread's rows and their first entries
  int lo[2], len[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t o0 = orow[h] & 0xFFFFu, o1 = orow[h] >> 16;
    lo[h] = o0 == kNoOff ? E : min((int)o0, E);
    const int hi = o1 == kNoOff ? E : min((int)o1, E);
    len[h] = max(hi - lo[h], 0);
  }
  uint32_t ent[2][kRowUnroll];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int j = 0; j < kRowUnroll; ++j) {
      ent[h][j] = kNoOff << 16;  // a sink with count 0 where the row has no entry j
      if (j < len[h]) ent[h][j] = entb[lo[h] + j];
    }
  }
  float rr[M][2];
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) rr[m][h] = V.d[m].P.R[row0 + min(tid + kBlock * h, nr - 1)];
  }
  // ---- each mission's window of v(t + 1) and own old values, straight to LDS
  int64_t wbase = 0;
  int wn = 0, wcols = P.nx;
  if (t + 1 < P.nt) {
    const BlockWin bw = block_window(P, t, c0, nst, P.narrow != 0);
    wbase = bw.base;
    wcols = bw.cols;
    wn = bw.rows * bw.cols;  // <= win_rows * nx = win
  }
  // [M][win + 1]: each mission's window, then a slot holding 0.0 (set once by
  // the kernel) that sink entries and a row's missing entries read
  const int wstride = win + 1;
  double *vwin0 = sm + kRowQ + 8;        // after Q and the block_max slots
  double *vself0 = vwin0 + M * wstride;  // [M][S]
  {
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!(live >> m & 1)) continue;  // uniform
      const char *src = reinterpret_cast<const char *>(vin(m) + wbase);
      char *dst = reinterpret_cast<char *>(vwin0 + m * wstride);
      if (wcols == P.nx) {  // whole rows: one contiguous range
        for (int j = wave * 64; j < 2 * wn; j += kBlock) {
          if (j + lane < 2 * wn)
            __builtin_amdgcn_global_load_lds((gptr_t)(src + 4 * (size_t)(j + lane)), (lptr_t)(dst + 4 * (size_t)j),
                                             4, 0, 0);
        }
      } else {  // a few columns of each row: a wave per row
        const int nrow = wn / wcols;
        for (int r = wave; r < nrow; r += kBlock / 64) {
          const char *srow = src + 8 * (size_t)r * P.nx;
          char *drow = dst + 8 * (size_t)r * wcols;
          for (int j = 0; j < 2 * wcols; j += 64)
            if (j + lane < 2 * wcols)
              __builtin_amdgcn_global_load_lds((gptr_t)(srow + 4 * (size_t)(j + lane)),
                                               (lptr_t)(drow + 4 * (size_t)j), 4, 0, 0);
        }
      }
      src = reinterpret_cast<const char *>(vin(m) + s0);
      dst = reinterpret_cast<char *>(vself0 + m * P.states_per_wg);
      for (int j = wave * 64; j < 2 * nst; j += kBlock) {
        if (j + lane < 2 * nst)
          __builtin_amdgcn_global_load_lds((gptr_t)(src + 4 * (size_t)(j + lane)), (lptr_t)(dst + 4 * (size_t)j), 4,
                                           0, 0);
      }
    }
  }
  prefetch();  // the next block's row offsets
  wait_vm();   // entries, rewards, this wave's copies (and the prefetch, in flight alongside)
  __syncthreads();  // every wave's copies
  const int qstride = P.na | 1;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    dres[m] = 0.0;
    if (!(live >> m & 1)) continue;
    const double *vw = vwin0 + m * wstride;
    // count x v(window index), a sink (index kNoOff) or a missing entry (count
    // 0, index kNoOff) reading the zero slot: acc + 0.0 is acc, and acc, a sum
    // from +0.0, is never -0.0, so every sum is the skipping sum's bit for bit
    const uint32_t wz = (uint32_t)win;
    double acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      acc[h] = 0.0;
      if constexpr (M == 1) {  // the row's window values read together, then summed
        double x[kRowUnroll];
#pragma unroll
        for (int j = 0; j < kRowUnroll; ++j) x[j] = vw[min(ent[h][j] >> 16, wz)];
#pragma unroll
        for (int j = 0; j < kRowUnroll; ++j) acc[h] += (double)(ent[h][j] & 0xFFFFu) * x[j];
      } else {  // two at a time (several missions' registers: reading more together spills)
#pragma unroll
        for (int j = 0; j < kRowUnroll; j += 2) {
          uint32_t e0 = ent[h][j], e1 = ent[h][j + 1];
          asm volatile("" : "+v"(e0), "+v"(e1));  // decoded per mission
          const double x0 = vw[min(e0 >> 16, wz)], x1 = vw[min(e1 >> 16, wz)];
          acc[h] += (double)(e0 & 0xFFFFu) * x0;
          acc[h] += (double)(e1 & 0xFFFFu) * x1;
        }
      }
      for (int k = kRowUnroll; k < len[h]; ++k) {  // the rest of a long row
        const uint32_t e = entb[lo[h] + k];
        acc[h] += (double)(e & 0xFFFFu) * vw[min(e >> 16, wz)];
      }
    }
    __syncthreads();  // the previous readers of qbuf
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = tid + kBlock * h;
      if (r < nr) qbuf[r + (qstride - P.na) * (r / P.na)] = (double)rr[m][h] + acc[h] * V.d[m].P.inv_nr;
    }
    __syncthreads();
    if (tid < nst) {
      int besta;
      const double best = first_max(qbuf + tid * qstride, P.na, besta);
      vout(m)[s0 + tid] = best;
      dres[m] = fabs(best - vself0[m * P.states_per_wg + tid]);
    }
  }
  // Every copy into LDS was waited for before the first barrier; what may be
  // in flight now is the block's value stores, which no later block of this
  // sweep reads (it reads the other buffer): only the LDS readers must be done.
  __syncthreads();
}

template <int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(M == 1 ? 8 : 7, 8))) void k_vi_sweep_rows(
    const MultiVI V, int t_hi, int win, double *wg_res)
{
  extern __shared__ double sm[];
  int live = 0, odd = 0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const VIState *st = V.d[m].st;
    live |= (st->done == 0) << m;
    odd |= (st->sweeps & 1) << m;
  }
  live = __builtin_amdgcn_readfirstlane(live);
  odd = __builtin_amdgcn_readfirstlane(odd);
  if (!live) return;  // every mission has converged
  // each mission's zero slot after its window (read after a block's first barrier)
  if (threadIdx.x < M) sm[kRowQ + 8 + threadIdx.x * (win + 1) + win] = 0.0;
  double d[M], dres[M];
#pragma unroll
  for (int m = 0; m < M; ++m) d[m] = 0.0;
  // the blocks of this workgroup, as for_blocks walks them, with the next
  // block's row offsets loaded during the current block
  const VIParams &P = V.d[0].P;
  const int bpl = P.blocks_per_layer;
  const int t_lo = min(P.t_lo, t_hi);
  const int b0 = t_lo * bpl;
  const int nb = (t_hi - t_lo) * bpl;
  const int x = (int)blockIdx.x % kXcds, nslot = (int)gridDim.x / kXcds;
  const int b_end = b0 + (int)((int64_t)nb * (x + 1) / kXcds);
  int b = b0 + (int)((int64_t)nb * x / kXcds) + (int)blockIdx.x / kXcds;
  if (b < b_end) {
    const int gq = nslot / bpl, gr = nslot % bpl;
    int t = b / bpl, c = b - t * bpl;
    RowSpan span = block_span(P, t, c * P.states_per_wg);
    uint32_t orow[2];
    load_row_offsets(P, t, c * P.states_per_wg, orow);
    for (; b < b_end; b += nslot) {
      int tn = t + gq, cn = c + gr;
      if (cn >= bpl) {
        cn -= bpl;
        ++tn;
      }
      const bool more = (int64_t)b + nslot < b_end;
      RowSpan nxt{0, 0};
      if (more) nxt = block_span(P, tn, cn * P.states_per_wg);
      uint32_t onext[2] = {kNoOff | kNoOff << 16, kNoOff | kNoOff << 16};
      vi_block_rows<M>(
          V, live, odd, t, c * P.states_per_wg, span, orow,
          [&] {
            if (more) load_row_offsets(P, tn, cn * P.states_per_wg, onext);
          },
          sm, win, dres);
#pragma unroll
      for (int m = 0; m < M; ++m) d[m] = fmax(d[m], dres[m]);
      t = tn;
      c = cn;
      span = nxt;
      orow[0] = onext[0];
      orow[1] = onext[1];
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double mx = block_max(d[m], sm + kRowQ);
    if (threadIdx.x == 0) wg_res[(int64_t)blockIdx.x * M + m] = mx;
  }
}

// Close the sweep of each mission (block m), as the batched close.
__global__ __launch_bounds__(kCloseBlock) void k_vi_close_missions(const MultiVI V, int grid, const double *wg_res,
                                                                    double tol)
{
  __shared__ double wmax[kCloseBlock / 64];
  const int i = blockIdx.x;
  VIState *st = V.d[i].st;
  if (st->done) return;
  double m = 0.0;
  for (int w = threadIdx.x; w < grid; w += kCloseBlock) m = fmax(m, wg_res[(int64_t)w * V.m + i]);
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

__global__ __launch_bounds__(kBlock) void k_vi_finish_missions(const MultiVI V, mdp_vi_stats *out)
{
  const int i = blockIdx.y;
  const BatchVIDesc &d = V.d[i];
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
  const int64_t nb = (int64_t)std::max(t_hi - P.t_lo, 0) * P.blocks_per_layer;
  const int grid = vi_grid(nb, std::min(P.n_wg, kViGridMax));
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
  const int grid = vi_grid(P.n_blocks, kViGridMax);
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

template <int M>
static hipError_t sweep_rows_t(const MultiVI &V, int t_hi, double *wg_res, double tol, hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_vi_sweep_rows<M>, attr);
  if (e != hipSuccess) return e;
  const VIParams &P = V.d[0].P;
  const int win = P.win_rows * P.nx;
  const size_t lds = ((size_t)kRowQ + 8 + (size_t)M * (win + 1 + P.states_per_wg)) * 8;
  const int64_t nb = (int64_t)t_hi * P.blocks_per_layer;
  const int grid = vi_grid(nb, kViGridMax);
  hipLaunchKernelGGL(k_vi_sweep_rows<M>, dim3(grid), dim3(kBlock), lds, s, V, t_hi, win, wg_res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_vi_close_missions, dim3(M), dim3(kCloseBlock), 0, s, V, grid, (const double *)wg_res, tol);
  return hipGetLastError();
}

template <int M>
static hipError_t sweep_missions_t(const MultiVI &V, int t_hi, double *wg_res, double tol, hipStream_t s)
{
  static bool attr = false;
  hipError_t e = allow_lds((const void *)k_vi_sweep_missions<M>, attr);
  if (e != hipSuccess) return e;
  const VIParams &P = V.d[0].P;
  const int win = P.win_rows * P.nx;
  const size_t lds = ((size_t)mvi_chunk(M) + 8 + (size_t)M * (win + P.states_per_wg)) * 8;
  const int64_t nb = (int64_t)t_hi * P.blocks_per_layer;
  const int grid = vi_grid(nb, kViGridMax);
  hipLaunchKernelGGL((k_vi_sweep_missions<M>), dim3(grid), dim3(kBlock), lds, s, V, t_hi, win, wg_res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_vi_close_missions, dim3(M), dim3(kCloseBlock), 0, s, V, grid, (const double *)wg_res, tol);
  return hipGetLastError();
}

hipError_t launch_vi_sweep_missions(const MultiVI &V, int t_hi, double *wg_res, double tol, hipStream_t s)
{
  const bool packed = V.d[0].P.ent != nullptr && V.d[0].P.win_rows > 0;
  switch (V.m) {
    case 1: return packed ? sweep_rows_t<1>(V, t_hi, wg_res, tol, s) : sweep_missions_t<1>(V, t_hi, wg_res, tol, s);
    case 2: return packed ? sweep_rows_t<2>(V, t_hi, wg_res, tol, s) : sweep_missions_t<2>(V, t_hi, wg_res, tol, s);
    case 3: return packed ? sweep_rows_t<3>(V, t_hi, wg_res, tol, s) : sweep_missions_t<3>(V, t_hi, wg_res, tol, s);
    default: return hipErrorInvalidValue;
  }
}

// Packed entries of the blocks of layers [t_lo, nt): one workgroup per block
// (grid-stride), the window of each block exactly as the fused sweep stages it.
__global__ __launch_bounds__(kBlock) void k_compact(const VIParams P, uint32_t *ent, uint16_t *roff, int t_lo)
{
  const int64_t nb = (int64_t)(P.nt - t_lo) * P.blocks_per_layer;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int t = t_lo + (int)(b / P.blocks_per_layer);
    const int c0 = (int)(b % P.blocks_per_layer) * P.states_per_wg;
    const int nst = min(P.states_per_wg, P.nc - c0);
    const int64_t row0 = ((int64_t)t * P.nc + c0) * P.na;
    const int64_t eb = min(max(P.row_ptr[row0], (int64_t)0), P.cap);
    const int64_t ee = min(max(P.row_ptr[row0 + (int64_t)nst * P.na], eb), P.cap);
    BlockWin bw{0, 0, 1};
    if (t + 1 < P.nt) bw = block_window(P, t, c0, nst, P.narrow != 0);
    const int64_t jw0 = (bw.base - (int64_t)(t + 1) * P.nc) / P.nx;
    const int64_t iw0 = (bw.base - (int64_t)(t + 1) * P.nc) - jw0 * P.nx;
    for (int64_t e = eb + threadIdx.x; e < ee; e += kBlock) {
      const int64_t rel = (int64_t)P.col[e] - (int64_t)(t + 1) * P.nc;  // state of layer t+1, or a sink
      uint32_t code = 0xFFFFu;
      if (t + 1 < P.nt && rel >= 0 && rel < P.nc) {
        const int rj = (int)rel / P.nx;  // a cell of the layer: 32-bit division
        const int r = rj - (int)jw0, k = (int)rel - rj * P.nx - (int)iw0;
        if (r >= 0 && r < bw.rows && k >= 0 && k < bw.cols) code = (uint32_t)(r * bw.cols + k);
      }
      ent[e] = code << 16 | (uint32_t)P.cnt[e];
    }
    const int64_t rb = P.row_ptr[row0];  // the block's first entry (offsets below 2^16 by the host's check)
    for (int r = threadIdx.x; r < nst * P.na; r += kBlock) roff[row0 + r] = (uint16_t)(P.row_ptr[row0 + r] - rb);
  }
}

hipError_t launch_compact(const VIParams &P, uint32_t *ent, uint16_t *roff, int t_lo, hipStream_t s)
{
  const int64_t nb = (int64_t)std::max(P.nt - t_lo, 0) * P.blocks_per_layer;
  if (nb == 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(nb, 16384);
  hipLaunchKernelGGL(k_compact, dim3(grid), dim3(kBlock), 0, s, P, ent, roff, t_lo);
  return hipGetLastError();
}

hipError_t launch_vi_finish_missions(const MultiVI &V, mdp_vi_stats *out, hipStream_t s)
{
  hipLaunchKernelGGL(k_vi_finish_missions, dim3(256, V.m), dim3(kBlock), 0, s, V, out);
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
