// Sparse-MDP build kernels for gfx950 (Alg. 1 and Alg. 2 of the paper,
// redesigned): one workgroup owns a tile of cells at one decision layer and
// all N_a actions of those cells, and walks the realizations in chunks.
//
//   phase A  (lane = realization): velocity synthesis u = ubar + sum_k mu_k phi_k
//            and the cell-unit position px = fma(u, dt/dx, i + 1/2) once per
//            (cell, realization), reused by every action. The coefficient
//            loads mu[t][k][r] are contiguous across lanes.
//   phase B  (lane = (cell, action) row): X = px + Hx[a], i' = floor(X), and a
//            private LDS counter per sub-grid bin. Counters are laid out
//            [bin][lane], so the 64 lanes of a wave always hit 64 distinct
//            banks whatever bins they land in; with 16-bit counters two rows
//            (lanes l and l + hw, hw = words per bin) share one word.
//   compaction (lane = row): bins in ascending order become CSR columns of
//            layer t+1 (out-of-domain, obstacle and beyond-horizon landings merge
//            into DEAD, the target into TARGET), the expected reward of every
//            mission is formed from the per-bin counts in fp64, and the entries
//            are packed into the workgroup's staging block.
// A one-block scan turns the per-workgroup entry counts into global offsets and
// a copy kernel writes row_ptr / col / cnt.
#include <math.h>

#include "mdp_internal.h"

namespace mdpk {

__device__ inline uint32_t wave_incl_scan(uint32_t x)
{
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over the 256 threads of a workgroup. sh: 4 words of LDS.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t *sh, uint32_t &total)
{
  const uint32_t inc = wave_incl_scan(x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint32_t v = sh[w];
    pre += (w < wave) ? v : 0u;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
}

__device__ inline unsigned long long block_sum_u64(unsigned long long x, unsigned long long *sh)
{
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  unsigned long long tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) tot += sh[w];
  __syncthreads();
  return tot;
}

// floor(x) converted to int in one VALU op (exact for |x| < 2^31).
__device__ inline int cvt_floor(float x)
{
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Atomic add to the 32-bit LDS word at byte address `addr`.
__device__ inline void lds_add(int addr, uint32_t v)
{
  lds_u32 *p = (lds_u32 *)(uintptr_t)(uint32_t)addr;
  (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// a * b + c on 24-bit signed operands in one VALU op.
__device__ inline int mad_i24(int a, int b, int c)
{
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// a * b + c with a wave-uniform b taken straight from a scalar register.
__device__ inline int mad_i24_s(int a, int b, int c)
{
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

__device__ inline uint64_t pack_entry(int32_t col, uint32_t cnt)
{
  return (uint64_t)(uint32_t)col | ((uint64_t)cnt << 32);
}

// Where one tile's outputs go. row_nnz/row_off are indexed from row_base for
// lane 0 of the tile; the staged entries go to `stage` when it is set, else to
// a slot bump-allocated from `pool` (recorded in *base_out, -1 on overflow).
struct TileOut {
  uint32_t *row_nnz, *row_off;
  int64_t row_base;
  uint64_t *stage;
  uint32_t *total_out;
  uint64_t *pool;
  unsigned long long *pool_top;
  int64_t pool_cap;
  int64_t *base_out;
};

// One tile of cells at layer t, every action of those cells, every realization.
// POOL: entries go to a bump-allocated pool slot instead of O.stage.
template <int KMAX, bool PACK16, bool NEAR, bool POOL, bool SWEPT = false, bool PAIRS = false, typename PT>
__device__ void build_tile(const PT &P, const int t, const int tile, BuildState *bst,
                           const TileOut &O, uint32_t *lds)
{
  const int HW = P.hw;                              // words per bin (power of 2)
  const int sstr = 2 * P.rch + 4;                   // floats per staged cell (padded)
  uint32_t *hist = lds;                             // [nbins][HW]; with SWEPT, bin nsg holds swept-path DEAD
  float *stage = reinterpret_cast<float *>(lds + P.nbins * HW);
  float *tab = stage + P.cells_per_tile * sstr;     // Hx[kMaxA], Hy[kMaxA]
  uint32_t *red = reinterpret_cast<uint32_t *>(tab + 2 * kMaxA);  // 16 words

  const int tid = threadIdx.x;
  const int c0 = tile * P.cells_per_tile;
  const int ncell = min(P.cells_per_tile, P.nc - c0);
  const int nc = P.nc;
  __syncthreads();  // LDS may still be read by the previous tile of a persistent loop

  // ---- this lane's row (cell cl of the tile, action a)
  const int cl = tid / P.na;
  const int a = tid - cl * P.na;
  const bool lane_row = tid < P.row_lanes && cl < ncell;
  const int c = c0 + (lane_row ? cl : 0);
  const int ci = c % P.nx, cj = c / P.nx;
  const float hxa = P.tab[a];
  const float hya = P.tab[kMaxA + a];
  if (tid < P.na) {
    tab[tid] = hxa;
    tab[kMaxA + tid] = hya;
  }
  const bool is_target = (ci == P.ti && cj == P.tj);
  const bool is_obst = P.mask != nullptr && P.mask[(size_t)t * nc + c] != 0;
  const bool sampled = lane_row && !is_target && !is_obst;

  for (int w = tid; w < P.nbins * HW; w += kBlock) hist[w] = 0u;
  // Swept-path test: only rows with an obstacle cell at t+1 inside their
  // sub-grid (other than their own cell) can have a blocked path.
  bool swept_row = false;
  const uint8_t *mask1 = (SWEPT && P.mask != nullptr) ? P.mask + (size_t)(t + 1) * nc : nullptr;
  if (SWEPT && mask1 != nullptr && sampled) {
    for (int dj = -P.hy; dj <= P.hy; ++dj)
      for (int di = -P.hx; di <= P.hx; ++di) {
        const int a2 = ci + di, b2 = cj + dj;
        if ((di | dj) != 0 && a2 >= 0 && a2 < P.nx && b2 >= 0 && b2 < P.ny && mask1[(size_t)b2 * P.nx + a2] != 0)
          swept_row = true;
      }
  }

  // word of bin (iy - cj + hy, ix - ci + hx) = (iy*W + ix)*HW + base
  const int col_l = tid & (HW - 1);
  const uint32_t inc = (PACK16 && (tid & HW)) ? 0x10000u : 1u;
  // byte address in LDS of this lane's counter for bin (iy*W + ix) - offset:
  // the dynamic allocation starts right after the kernel's static LDS
  const int base4 = (int)__builtin_amdgcn_groupstaticsize() +
                    (((P.hy - cj) * P.W + (P.hx - ci)) * HW + col_l) * 4;
  const int HW4 = HW * 4;
  const int W = P.W;
  // The row's counters for the compaction: column row_col, 16-bit half
  // row_shift (lanes own rows, two rows a word with 16-bit counters).
  int row_col = col_l;
  int row_shift = (PACK16 && (tid & HW)) ? 16 : 0;
  // PAIRS (16-bit counters): in the landing loop a lane owns the two rows of
  // a pair of actions of one cell, both counters in one word (low: the
  // pair's first action; the pair's column: pairs whose actions share Hx
  // bitwise first, cell by cell, then the others), and one of kBlock / HW
  // parts of each chunk's realizations. The lanes take (pair, part) jobs with
  // every part of the shared-Hx pairs first, so whole waves hold only such
  // pairs and compute the x add, floor and column offset once for both rows;
  // the jobs of the other pairs take the last lanes.
  const int npc = P.na >> 1, nreal = P.n_real_pairs, npseudo = npc - nreal;
  const int nrl = P.cells_per_tile * nreal, nps = P.cells_per_tile * npseudo;  // pair columns of each kind
  auto pair_lane = [&](int cell, int q) { return q < nreal ? cell * nreal + q : nrl + cell * npseudo + (q - nreal); };
  int pr_cell = 0, pr_q = 0, pr_col = 0, pr_part = 0;
  const int pr_nparts = kBlock / HW;
  if constexpr (PAIRS) {
    const int rp = P.row_pair[a];
    row_col = pair_lane(cl, rp >> 1);
    row_shift = (rp & 1) ? 16 : 0;
    if (tid < nrl * pr_nparts) {  // a part of a shared-Hx pair
      pr_col = tid % nrl;
      pr_part = tid / nrl;
      pr_cell = pr_col / nreal;
      pr_q = pr_col - pr_cell * nreal;
    } else if (tid < (nrl + nps) * pr_nparts) {  // a part of another pair
      const int j = tid - nrl * pr_nparts;
      pr_col = nrl + j % nps;
      pr_part = j / nps;
      pr_cell = (j % nps) / npseudo;
      pr_q = nreal + (j % nps) - pr_cell * npseudo;
    } else {
      pr_cell = P.cells_per_tile;  // no pair
    }
  }

  const int rmask = P.rch - 1;
  const int rlane = tid & rmask;
  const int qg = __builtin_amdgcn_readfirstlane(tid / P.rch);  // uniform per wave (rch >= 64)
  const int nqg = kBlock / P.rch;
  const size_t tm_off = (size_t)P.mean_tstride * t;
  const size_t tp_off = (size_t)P.mode_tstride * t;
  const float *mu_t = P.mu + (size_t)t * P.K * P.nr;

  uint32_t near_cnt = 0, esc_cnt = 0;
  // Coefficients of this lane's realization in chunk r0. Coefficients beyond K
  // are zero, so their fma(0, phi, u) terms return u exactly and the landing
  // arithmetic is the K-term sum; loads are clamped to mode K-1 and to the last
  // realization (every load in bounds) instead of branching.
  // K is KMAX or KMAX - 1 (the kernel is compiled for even mode bounds), so
  // only the last slot can be a zero term. Each mode's row is a uniform base
  // address plus the lane's 32-bit offset: no per-mode vector address
  // arithmetic.
  const bool last_mode = P.K == KMAX;
  auto load_mu = [&](int r0, float *m) {
    const uint32_t rb = 4u * (uint32_t)min(r0 + rlane, P.nr - 1);  // byte offset of the lane's realization
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const char *mk = reinterpret_cast<const char *>(mu_t + (size_t)(k < KMAX - 1 ? k : P.K - 1) * P.nr);
      const float val = *reinterpret_cast<const float *>(mk + rb);
      m[k] = (k < KMAX - 1 || last_mode) ? val : 0.0f;
    }
  };
  float m[KMAX];  // coefficients of the current chunk
  load_mu(0, m);
  __syncthreads();

  // PAIRS: this lane's pair of rows (the action tables are in LDS now)
  static_assert(!PAIRS || (PACK16 && !NEAR && !SWEPT), "paired landing loop: 16-bit counters only");
  bool pr_live = false, pr_real = false;
  int pr_base4 = 0;
  float pr_hx1 = 0.0f, pr_hx2 = 0.0f, pr_hy1 = 0.0f, pr_hy2 = 0.0f;
  const int WHW4 = W * HW4;
  if constexpr (PAIRS) {
    if (pr_cell < ncell) {
      const int pc = c0 + pr_cell;
      const int pci = pc % P.nx, pcj = pc / P.nx;
      pr_live = !(pci == P.ti && pcj == P.tj) && !(P.mask != nullptr && P.mask[(size_t)t * nc + pc] != 0);
      const int a1 = P.pair_a[2 * pr_q], a2 = P.pair_a[2 * pr_q + 1];
      pr_hx1 = tab[a1];
      pr_hx2 = tab[a2];
      pr_hy1 = tab[kMaxA + a1];
      pr_hy2 = tab[kMaxA + a2];
      pr_real = pr_q < nreal;
      pr_base4 = (int)__builtin_amdgcn_groupstaticsize() + (((P.hy - pcj) * W + (P.hx - pci)) * HW + pr_col) * 4;
    }
  }

  for (int r0 = 0; r0 < P.nr; r0 += P.rch) {
    const int nloc = min(P.rch, P.nr - r0);
    // ---------------- phase A: lane = realization
    {
      const bool rv = rlane < nloc;
      for (int q = qg; q < ncell; q += nqg) {
        const int cq = c0 + q;
        const int qi = cq % P.nx, qj = cq / P.nx;
        const bool q_skip = (qi == P.ti && qj == P.tj) ||
                            (P.mask != nullptr && P.mask[(size_t)t * nc + cq] != 0);
        if (q_skip) continue;
        float u = P.ubar[tm_off + cq];
        float v = P.vbar[tm_off + cq];
        const float *pu = P.phiu + tp_off + cq;
        const float *pv = P.phiv + tp_off + cq;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          const size_t ko = (size_t)min(k, P.K - 1) * nc;
          u = __builtin_fmaf(m[k], pu[ko], u);
          v = __builtin_fmaf(m[k], pv[ko], v);
        }
        float px = __builtin_fmaf(u, P.lam_x, (float)qi + 0.5f);
        float py = __builtin_fmaf(v, P.lam_y, (float)qj + 0.5f);
        if (rv && !(fabsf(u) <= P.usafe && fabsf(v) <= P.vsafe)) {
          // Possible escape: check every action exactly (a non-finite flow
          // counts as escaping with every action).
          uint32_t n = 0;
          if (!isfinite(u) || !isfinite(v)) {
            n = (uint32_t)P.na;
          } else {
            for (int aa = 0; aa < P.na; ++aa) {
              const float X = px + tab[aa];
              const float Y = py + tab[kMaxA + aa];
              const int di = (int)floorf(X) - qi, dj = (int)floorf(Y) - qj;
              n += (abs(di) > P.hx || abs(dj) > P.hy) ? 1u : 0u;
            }
          }
          if (n) {  // the model is invalid anyway; keep the histogram in bounds
            esc_cnt += n;
            px = (float)qi + 0.5f;
            py = (float)qj + 0.5f;
          }
        }
        *reinterpret_cast<float2 *>(stage + q * sstr + 2 * rlane) = make_float2(px, py);
      }
    }
    __syncthreads();
    // ---------------- phase B: lane = (cell, action) row, or (PAIRS) a pair of rows
    if constexpr (PAIRS) {
      if (pr_live) {
        const float4 *st4 = reinterpret_cast<const float4 *>(stage + pr_cell * sstr);
        const float2 *st2 = reinterpret_cast<const float2 *>(stage + pr_cell * sstr);
        const int n4 = nloc >> 2;  // groups of four realizations; this part's share of them
        const int g0 = n4 * pr_part / pr_nparts, g1 = n4 * (pr_part + 1) / pr_nparts;
        const bool tail = pr_part == pr_nparts - 1;  // the chunk's last (nloc mod 4) realizations
        // Both rows of the pair share the x add, floor and column offset when
        // their Hx agree bitwise; a wave whose pairs all do takes that loop,
        // the wave holding the other pairs computes both (a uniform branch).
        const bool wave_shared = __ballot(!pr_real) == 0;
        // two register sets alternate, the next group loaded before the
        // current group's counter updates (no prefetch past this part's groups)
        auto group_loop = [&](auto &&pbin) {
          auto four = [&](const float4 &X0, const float4 &X1) {
            pbin(X0.x, X0.y);
            pbin(X0.z, X0.w);
            pbin(X1.x, X1.y);
            pbin(X1.z, X1.w);
          };
          int g = g0;
          if (g < g1) {
            float4 A0 = st4[2 * g], A1 = st4[2 * g + 1];
            for (; g + 4 < g1; g += 4) {  // four groups an iteration, two register sets
              float4 B0 = st4[2 * g + 2], B1 = st4[2 * g + 3];
              four(A0, A1);
              A0 = st4[2 * g + 4];
              A1 = st4[2 * g + 5];
              four(B0, B1);
              B0 = st4[2 * g + 6];
              B1 = st4[2 * g + 7];
              four(A0, A1);
              A0 = st4[2 * g + 8];
              A1 = st4[2 * g + 9];
              four(B0, B1);
            }
            for (; g + 2 < g1; g += 2) {
              const float4 B0 = st4[2 * g + 2], B1 = st4[2 * g + 3];
              four(A0, A1);
              A0 = st4[2 * g + 4];
              A1 = st4[2 * g + 5];
              four(B0, B1);
            }
            if (g + 1 < g1) {
              const float4 B0 = st4[2 * g + 2], B1 = st4[2 * g + 3];
              four(A0, A1);
              four(B0, B1);
            } else {
              four(A0, A1);
            }
          }
          if (tail)
            for (int rr = n4 * 4; rr < nloc; ++rr) {
              const float2 pp = st2[rr];
              pbin(pp.x, pp.y);
            }
        };
        if (wave_shared) {
          group_loop([&](float px, float py) {
            const int xb = mad_i24_s(cvt_floor(px + pr_hx1), HW4, pr_base4);
            lds_add(mad_i24_s(cvt_floor(py + pr_hy1), WHW4, xb), 1u);
            lds_add(mad_i24_s(cvt_floor(py + pr_hy2), WHW4, xb), 0x10000u);
          });
        } else {
          group_loop([&](float px, float py) {
            const int xb = mad_i24_s(cvt_floor(px + pr_hx1), HW4, pr_base4);
            const int xb2 = mad_i24_s(cvt_floor(px + pr_hx2), HW4, pr_base4);
            lds_add(mad_i24_s(cvt_floor(py + pr_hy1), WHW4, xb), 1u);
            lds_add(mad_i24_s(cvt_floor(py + pr_hy2), WHW4, xb2), 0x10000u);
          });
        }
      }
    } else if (sampled) {
      // Staged positions of this row's cell are read 4 realizations at a time;
      // the next group is loaded before the current group's counter updates.
      const float4 *st4 = reinterpret_cast<const float4 *>(stage + cl * sstr);
      const int n4 = nloc >> 2;
      // word of the swept-path DEAD bin (bin nsg) of this lane
      const int dead4 = (int)__builtin_amdgcn_groupstaticsize() + (P.nsg * HW + col_l) * 4;
      auto bin = [&](float px, float py) {
        const float X = px + hxa;
        const float Y = py + hya;
        const int ix = cvt_floor(X);
        const int iy = cvt_floor(Y);
        int addr = mad_i24_s(mad_i24_s(iy, W, ix), HW4, base4);
        if (SWEPT && swept_row && swept_blocked(mask1, P.nx, P.ny, ci, cj, ix, iy, X, Y)) addr = dead4;
        lds_add(addr, inc);
        if (NEAR)
          near_cnt += ((fabsf(X - rintf(X)) < P.eps_x) || (fabsf(Y - rintf(Y)) < P.eps_y)) ? 1u : 0u;
      };
      // Two register sets alternate; a prefetch may read up to 16 bytes past
      // this cell's padded block, which stays inside the LDS allocation (the
      // next cell's block or the action table) and is never used.
      int g = 0;
      if (n4 > 0) {
        float4 A0 = st4[0], A1 = st4[1];
        for (; g + 2 <= n4; g += 2) {
          const float4 B0 = st4[2 * g + 2], B1 = st4[2 * g + 3];
          bin(A0.x, A0.y);
          bin(A0.z, A0.w);
          bin(A1.x, A1.y);
          bin(A1.z, A1.w);
          A0 = st4[2 * g + 4];
          A1 = st4[2 * g + 5];
          bin(B0.x, B0.y);
          bin(B0.z, B0.w);
          bin(B1.x, B1.y);
          bin(B1.z, B1.w);
        }
        if (g < n4) {
          bin(A0.x, A0.y);
          bin(A0.z, A0.w);
          bin(A1.x, A1.y);
          bin(A1.z, A1.w);
        }
      }
      const float2 *st2 = reinterpret_cast<const float2 *>(stage + cl * sstr);
      for (int rr = n4 * 4; rr < nloc; ++rr) {
        const float2 pp = st2[rr];
        bin(pp.x, pp.y);
      }
    }
    __syncthreads();
    if (r0 + P.rch < P.nr) load_mu(r0 + P.rch, m);
  }

  // ---------------- diagnostics
  {
    unsigned long long *red64 = reinterpret_cast<unsigned long long *>(red);
    const unsigned long long e = block_sum_u64(esc_cnt, red64);
    const unsigned long long nr_ = block_sum_u64(NEAR ? near_cnt : 0u, red64);
    const unsigned long long smp = block_sum_u64(sampled ? (unsigned long long)P.nr : 0ull, red64);
    if (tid == 0) {
      if (e) atomicAdd(&bst->n_escape, e);
      if (nr_) atomicAdd(&bst->n_near, nr_);
      atomicAdd(&bst->samples, smp);
    }
  }

  // ---------------- compaction, pass 1: entries and rewards of the row
  const int32_t ns = P.nt * nc;
  const int32_t DEAD = ns, TARGET = ns + 1;
  const size_t m1 = (size_t)(t + 1) * nc;
  const bool last_layer = (t + 1 == P.nt);
  const int jf = a / P.n_head;
  const double F = P.f_max * (double)(jf + 1) / (double)P.n_speed;
  const double e_a = P.c_f * F * F;
  const double g_s = (P.gbar != nullptr && lane_row) ? (double)P.gbar[(size_t)t * nc + c] : 0.0;
  const int shift = row_shift;

  uint32_t nnz = 0, dead = 0, tgt = 0, nstate = 0;
  double gsum = 0.0;  // sum over state and target landings of count * gbar(s')
  if (sampled) {
    int b = 0;
    for (int dj = -P.hy; dj <= P.hy; ++dj) {
      const int jp = cj + dj;
      for (int di = -P.hx; di <= P.hx; ++di, ++b) {
        const uint32_t wv = hist[b * HW + row_col];
        const uint32_t n = PACK16 ? ((wv >> shift) & 0xffffu) : wv;
        if (n == 0) continue;
        const int ip = ci + di;
        if (ip < 0 || ip >= P.nx || jp < 0 || jp >= P.ny) {
          dead += n;
          continue;
        }
        const int cp = jp * P.nx + ip;
        if (P.mask != nullptr && P.mask[m1 + cp] != 0) {
          dead += n;
        } else if (ip == P.ti && jp == P.tj) {
          tgt += n;
          if (P.gbar != nullptr) gsum += (double)n * (double)P.gbar[m1 + cp];
        } else if (last_layer) {
          dead += n;
        } else {
          ++nnz;
          nstate += n;
          if (P.gbar != nullptr) gsum += (double)n * (double)P.gbar[m1 + cp];
        }
      }
    }
    if (SWEPT) {  // samples whose path entered an obstacle at t+1
      const uint32_t wv = hist[P.nsg * HW + row_col];
      dead += PACK16 ? ((wv >> shift) & 0xffffu) : wv;
    }
    nnz += (dead ? 1u : 0u) + (tgt ? 1u : 0u);
  } else if (lane_row) {
    nnz = 1;
  }

  // ---------------- rewards (per-bin counts, fp64)
  if (lane_row) {
    const int64_t row = ((int64_t)t * nc + c) * P.na + a;
    const double inv = 1.0 / (double)P.nr;
    const double live = (double)(nstate + tgt);
    const double fixed = P.r_term * (double)tgt + P.r_out * (double)dead;
    for (int k = 0; k < P.nmiss; ++k) {
      const int m = P.miss[k];
      double Rm;
      if (is_target) {
        Rm = 0.0;
      } else if (is_obst) {
        Rm = P.r_out;
      } else {
        double s;
        if (m == MDP_MISSION_TIME)
          s = -P.dt * live + fixed;
        else if (m == MDP_MISSION_ENERGY)
          s = -e_a * P.dt * live + fixed;
        else
          s = (-e_a + 0.5 * P.c_r * g_s) * P.dt * live + 0.5 * P.c_r * P.dt * gsum + fixed;
        Rm = s * inv;
      }
      P.reward[(int64_t)k * P.rows + row] = (float)Rm;
    }
  }

  // ---------------- workgroup offsets
  uint32_t total;
  const uint32_t off = block_excl_scan(nnz, red, total);
  if (lane_row) {
    O.row_nnz[O.row_base + tid] = nnz;
    O.row_off[O.row_base + tid] = off;
  }
  if (tid == 0) *O.total_out = total;
  // Staging block: fixed per tile, or bump-allocated from the pool (a tile
  // that does not fit is recorded as -1 and writes nothing).
  uint64_t *blk = O.stage;
  if constexpr (POOL) {
    unsigned long long *bcast = reinterpret_cast<unsigned long long *>(red) + 2;
    if (tid == 0) {
      const unsigned long long b0 = atomicAdd(O.pool_top, (unsigned long long)total);
      const bool fits = (int64_t)(b0 + total) <= O.pool_cap;
      *O.base_out = fits ? (int64_t)b0 : -1;
      bcast[0] = fits ? b0 : ~0ull;
    }
    __syncthreads();
    blk = (bcast[0] != ~0ull) ? O.pool + bcast[0] : nullptr;
  }

  // ---------------- compaction, pass 2: write the row's entries
  if (lane_row && blk != nullptr) {
    uint64_t *out = blk + off;
    if (!sampled) {
      out[0] = pack_entry(is_target ? TARGET : DEAD, (uint32_t)P.nr);
    } else {
      uint32_t k = 0;
      int b = 0;
      for (int dj = -P.hy; dj <= P.hy; ++dj) {
        const int jp = cj + dj;
        for (int di = -P.hx; di <= P.hx; ++di, ++b) {
          const uint32_t wv = hist[b * HW + row_col];
          const uint32_t n = PACK16 ? ((wv >> shift) & 0xffffu) : wv;
          if (n == 0 || last_layer) continue;
          const int ip = ci + di;
          if (ip < 0 || ip >= P.nx || jp < 0 || jp >= P.ny) continue;
          const int cp = jp * P.nx + ip;
          if (P.mask != nullptr && P.mask[m1 + cp] != 0) continue;
          if (ip == P.ti && jp == P.tj) continue;
          out[k++] = pack_entry((int32_t)((t + 1) * nc + cp), n);
        }
      }
      if (dead) out[k++] = pack_entry(DEAD, dead);
      if (tgt) out[k++] = pack_entry(TARGET, tgt);
    }
  }
}

template <int KMAX, bool PACK16, bool NEAR, bool SWEPT, bool PAIRS>
__global__ __launch_bounds__(kBlock) void k_build(const BuildParams P, const SlabParams S)
{
  extern __shared__ __align__(16) uint32_t lds[];
  const int wg = blockIdx.x;
  const int tl = wg / P.tiles_per_layer;
  const int tile = wg - tl * P.tiles_per_layer;
  const int t = S.t0 + tl;
  TileOut O;
  O.row_nnz = S.row_nnz;
  O.row_off = S.row_off;
  O.row_base = ((int64_t)t * P.nc + (int64_t)tile * P.cells_per_tile) * P.na - S.row0;
  O.stage = S.stage + (int64_t)wg * S.wg_cap;
  O.total_out = S.wg_nnz + wg;
  O.pool = nullptr;
  O.pool_top = nullptr;
  O.pool_cap = 0;
  O.base_out = nullptr;
  build_tile<KMAX, PACK16, NEAR, false, SWEPT, PAIRS>(P, t, tile, S.st, O, lds);
}

// Action displacement tables into device memory (one thread per entry).
__global__ void k_fill_tab(const ActionTables T, float *tab)
{
  const int k = threadIdx.x;
  float x = 0.0f;
#pragma unroll
  for (int q = 0; q < 2 * kMaxA; ++q)
    if (q == k) x = (q < kMaxA) ? T.hx[q] : T.hy[q - kMaxA];
  if (k < 2 * kMaxA) tab[k] = x;
}

__global__ void k_build_init(BuildState *st, const int64_t *row_ptr_row0)
{
  if (threadIdx.x == 0) {
    st->n_escape = 0;
    st->n_near = 0;
    st->samples = 0;
    st->running_nnz = row_ptr_row0 ? *row_ptr_row0 : 0;
  }
}

// Exclusive scan of the per-workgroup entry counts of one pass (one block),
// in tiles of 1024 x kScanPer counts: read coalesced into LDS, kScanPer
// consecutive counts per thread, a block scan of the thread sums (lane
// shuffles within a wave, then the wave totals), the offsets written
// kScanPer consecutive ones per thread, the running total carried to the
// next tile.
constexpr int kScanPer = 8;
__global__ __launch_bounds__(1024) void k_scan_wg(const uint32_t *wg_nnz, int n, int64_t *wg_off,
                                                  BuildState *st, int64_t *row_ptr_end)
{
  __shared__ uint32_t cnt[1024 * kScanPer];
  __shared__ long long wsum[1024 / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long carry = st->running_nnz;
  for (int base = 0; base < n; base += 1024 * kScanPer) {
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const int k = base + i * 1024 + tid;
      cnt[i * 1024 + tid] = k < n ? wg_nnz[k] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanPer];
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      v[j] = cnt[tid * kScanPer + j];
      s += v[j];
    }
    long long x = s;  // inclusive scan of the thread sums within the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const long long y = __shfl_up(x, d, 64);
      x += lane >= d ? y : 0ll;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    long long before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 1024 / 64; ++w) {
      const long long tw = wsum[w];
      before += w < wave ? tw : 0ll;
      total += tw;
    }
    long long acc = carry + before + x - s;  // offset of this thread's first count
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      const int k = base + tid * kScanPer + j;
      if (k < n) wg_off[k] = acc;
      acc += v[j];
    }
    carry += total;
    __syncthreads();  // the tile's LDS reads before the next tile's writes
  }
  if (tid == 0) {
    st->running_nnz = carry;
    if (row_ptr_end) *row_ptr_end = carry;
  }
}

// row_ptr of the pass's rows and the staged entries -> CSR (capacity-checked).
__global__ __launch_bounds__(kBlock) void k_copy(const BuildParams P, const SlabParams S,
                                                  const ModelOut M)
{
  const int tid = threadIdx.x;
  const int wg = blockIdx.x;
  const int tl = wg / P.tiles_per_layer;
  const int tile = wg - tl * P.tiles_per_layer;
  const int t = S.t0 + tl;
  const int c0 = tile * P.cells_per_tile;
  const int ncell = min(P.cells_per_tile, P.nc - c0);
  const int64_t off = S.wg_off[wg];
  if (tid < ncell * P.na) {
    const int64_t row = ((int64_t)t * P.nc + c0) * P.na + tid;
    M.row_ptr[row] = off + S.row_off[row - S.row0];
  }
  const uint32_t n = S.wg_nnz[wg];
  const uint64_t *src = S.stage + (int64_t)wg * S.wg_cap;
  for (uint32_t k = tid; k < n; k += kBlock) {
    const int64_t d = off + k;
    if (d < M.capacity) {
      const uint64_t e = src[k];
      M.col[d] = (int32_t)(uint32_t)e;
      M.cnt[d] = (uint16_t)(e >> 32);
    }
  }
}

__global__ void k_build_finalize(BuildState *st, int64_t capacity, int n_slabs, int near_asked)
{
  if (threadIdx.x != 0) return;
  mdp_build_stats o;
  o.samples = (int64_t)st->samples;
  o.nnz = st->running_nnz;
  o.n_escape = (int64_t)st->n_escape;
  o.n_near_edge = near_asked ? (int64_t)st->n_near : -1;
  o.status = o.n_escape ? MDP_E_SUBGRID : (o.nnz > capacity ? MDP_E_CAPACITY : MDP_OK);
  o.n_slabs = n_slabs;
  st->out = o;
}

// Exact escape count without a histogram, for sub-grids too small to hold even
// the agent's own displacement (the model is then not built).
__global__ __launch_bounds__(kBlock) void k_escape_only(const BuildParams P, BuildState *st)
{
  const int nc = P.nc;
  const int64_t total = (int64_t)P.nt * nc * P.nr;
  unsigned long long n = 0, smp = 0;
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * kBlock) {
    const int r = (int)(id % P.nr);
    const int64_t tc = id / P.nr;
    const int c = (int)(tc % nc);
    const int t = (int)(tc / nc);
    const int ci = c % P.nx, cj = c / P.nx;
    if ((ci == P.ti && cj == P.tj) || (P.mask != nullptr && P.mask[(size_t)t * nc + c] != 0)) continue;
    float u = P.ubar[(size_t)P.mean_tstride * t + c];
    float v = P.vbar[(size_t)P.mean_tstride * t + c];
    for (int k = 0; k < P.K; ++k) {
      const float m = P.mu[((size_t)t * P.K + k) * P.nr + r];
      u = __builtin_fmaf(m, P.phiu[(size_t)P.mode_tstride * t + (size_t)k * nc + c], u);
      v = __builtin_fmaf(m, P.phiv[(size_t)P.mode_tstride * t + (size_t)k * nc + c], v);
    }
    const float px = __builtin_fmaf(u, P.lam_x, (float)ci + 0.5f);
    const float py = __builtin_fmaf(v, P.lam_y, (float)cj + 0.5f);
    for (int a = 0; a < P.na; ++a) {
      const float X = px + P.tab[a], Y = py + P.tab[kMaxA + a];
      const int di = (int)floorf(X) - ci, dj = (int)floorf(Y) - cj;
      n += (abs(di) > P.hx || abs(dj) > P.hy) ? 1ull : 0ull;
    }
    smp += P.na;
  }
  __shared__ unsigned long long sh[4];
  const unsigned long long tn = block_sum_u64(n, sh);
  const unsigned long long ts = block_sum_u64(smp, sh);
  if (threadIdx.x == 0) {
    if (tn) atomicAdd(&st->n_escape, tn);
    atomicAdd(&st->samples, ts);
  }
}

// Largest |u| and |v| over all synthesised velocities (bits of non-negative
// floats order like unsigned integers).
__global__ __launch_bounds__(kBlock) void k_max_speed(const BuildParams P, unsigned int *bits)
{
  const int nc = P.nc;
  const int64_t total = (int64_t)P.nt * nc * P.nr;
  float mu_ = 0.0f, mv = 0.0f;
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * kBlock) {
    const int r = (int)(id % P.nr);
    const int64_t tc = id / P.nr;
    const int c = (int)(tc % nc);
    const int t = (int)(tc / nc);
    float u = P.ubar[(size_t)P.mean_tstride * t + c];
    float v = P.vbar[(size_t)P.mean_tstride * t + c];
    for (int k = 0; k < P.K; ++k) {
      const float m = P.mu[((size_t)t * P.K + k) * P.nr + r];
      u = __builtin_fmaf(m, P.phiu[(size_t)P.mode_tstride * t + (size_t)k * nc + c], u);
      v = __builtin_fmaf(m, P.phiv[(size_t)P.mode_tstride * t + (size_t)k * nc + c], v);
    }
    mu_ = fmaxf(mu_, fabsf(u));
    mv = fmaxf(mv, fabsf(v));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    mu_ = fmaxf(mu_, __shfl_xor(mu_, d, 64));
    mv = fmaxf(mv, __shfl_xor(mv, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&bits[0], __float_as_uint(mu_));
    atomicMax(&bits[1], __float_as_uint(mv));
  }
}

// ------------------------------------------------------------------ batches
__global__ void k_batch_build_init(BatchBuildDesc *D, int n, unsigned int *counter,
                                   unsigned long long *pool_top)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMaxBuildLaunches) counter[i] = 0u;
  if (i == 0) *pool_top = 0ull;
  if (i < n) {
    BuildState *st = D[i].st;
    st->n_escape = 0;
    st->n_near = 0;
    st->samples = 0;
    st->running_nnz = 0;
    st->pad[0] = 0;  // pool overflow flag
  }
}

// Persistent build over every problem of a batch: workgroups take (problem,
// layer, tile) items from a shared counter until the list (sorted by cost,
// largest first) runs out; each item's entries go to a bump-allocated pool slot.
template <int KMAX, bool NEAR>
__global__ __launch_bounds__(kBlock) void k_build_batched(const BatchBuildDesc *D, const BatchItem *items,
                                                           int n_items, unsigned int *counter, uint64_t *pool,
                                                           unsigned long long *pool_top, int64_t pool_cap)
{
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_s);  // uniform: descriptor loads go scalar
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem w = load_const(items + it);
    // descriptor fields are read in place through the constant address space
    typedef const __attribute__((address_space(4))) BatchBuildDesc CDesc;
    CDesc &d = *(CDesc *)(uintptr_t)(D + w.inst);
    auto &P = d.P;
    const int64_t local = (int64_t)w.t * P.tiles_per_layer + w.tile;
    TileOut O;
    O.row_nnz = d.row_nnz;
    O.row_off = d.row_off;
    O.row_base = ((int64_t)w.t * P.nc + (int64_t)w.tile * P.cells_per_tile) * P.na;
    O.stage = nullptr;
    O.total_out = d.item_total + local;
    O.pool = pool;
    O.pool_top = pool_top;
    O.pool_cap = pool_cap;
    O.base_out = d.item_base + local;
    build_tile<KMAX, true, NEAR, true>(P, w.t, w.tile, d.st, O, lds);
  }
}

// Per problem (one block each): exclusive scan of its items' entry counts in
// row order, the end of row_ptr, the nnz total and the pool-overflow flag.
__global__ __launch_bounds__(1024) void k_batch_scan(BatchBuildDesc *D)
{
  BatchBuildDesc &d = D[blockIdx.x];
  __shared__ long long sh[1024];
  const int tid = threadIdx.x;
  const int64_t n = d.n_items;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = min(n, (int64_t)tid * per), hi = min(n, lo + per);
  long long s = 0;
  int over = 0;
  for (int64_t k = lo; k < hi; ++k) {
    s += d.item_total[k];
    over |= (d.item_base[k] < 0) ? 1 : 0;
  }
  over = __syncthreads_or(over);
  sh[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long y = (tid >= o) ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  long long acc = sh[tid] - s;
  for (int64_t k = lo; k < hi; ++k) {
    d.item_off[k] = acc;
    acc += d.item_total[k];
  }
  if (tid == 1023) {
    d.st->running_nnz = sh[1023];
    d.M.row_ptr[d.P.rows] = sh[1023];
    d.st->pad[0] = over;
  }
}

// Every item: row_ptr of its rows and its pool slot into the CSR (capacity-checked).
__global__ __launch_bounds__(kBlock) void k_batch_copy(const BatchBuildDesc *D, const BatchItem *items,
                                                        int n_items, const uint64_t *pool)
{
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const BatchItem w = items[it];
    const BatchBuildDesc &d = D[w.inst];
    const int64_t local = (int64_t)w.t * d.P.tiles_per_layer + w.tile;
    const int c0 = w.tile * d.P.cells_per_tile;
    const int ncell = min(d.P.cells_per_tile, d.P.nc - c0);
    const int64_t row0 = ((int64_t)w.t * d.P.nc + c0) * d.P.na;
    const int64_t off = d.item_off[local];
    const int64_t base = d.item_base[local];
    const uint32_t n = d.item_total[local];
    if (tid < ncell * d.P.na) d.M.row_ptr[row0 + tid] = off + d.row_off[row0 + tid];
    if (base >= 0) {
      for (uint32_t k = tid; k < n; k += kBlock) {
        const int64_t dst = off + k;
        if (dst < d.M.capacity) {
          const uint64_t e = pool[base + k];
          d.M.col[dst] = (int32_t)(uint32_t)e;
          d.M.cnt[dst] = (uint16_t)(e >> 32);
        }
      }
    }
  }
}

__global__ void k_batch_finalize(BatchBuildDesc *D, int n, mdp_build_stats *out)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BuildState *st = D[i].st;
  mdp_build_stats o;
  o.samples = (int64_t)st->samples;
  o.nnz = st->running_nnz;
  o.n_escape = (int64_t)st->n_escape;
  o.n_near_edge = D[i].near_asked ? (int64_t)st->n_near : -1;
  o.status = o.n_escape ? MDP_E_SUBGRID
                        : (st->pad[0] ? MDP_E_SCRATCH : (o.nnz > D[i].M.capacity ? MDP_E_CAPACITY : MDP_OK));
  o.n_slabs = 1;
  out[i] = o;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_fill_tab(const ActionTables &T, float *tab, hipStream_t s)
{
  hipLaunchKernelGGL(k_fill_tab, dim3(1), dim3(2 * kMaxA), 0, s, T, tab);
  return hipGetLastError();
}

hipError_t launch_build_init(BuildState *st, hipStream_t s)
{
  hipLaunchKernelGGL(k_build_init, dim3(1), dim3(64), 0, s, st, (const int64_t *)nullptr);
  return hipGetLastError();
}

hipError_t launch_build_init_from(BuildState *st, const int64_t *row_ptr_row0, hipStream_t s)
{
  hipLaunchKernelGGL(k_build_init, dim3(1), dim3(64), 0, s, st, row_ptr_row0);
  return hipGetLastError();
}

template <int KMAX, bool PACK16, bool NEAR, bool SWEPT, bool PAIRS = false>
static hipError_t launch_build_t(const BuildParams &P, const SlabParams &S, size_t lds, hipStream_t s)
{
  auto kern = k_build<KMAX, PACK16, NEAR, SWEPT, PAIRS>;
  static bool attr_set = false;  // raise the dynamic-LDS limit once per instantiation
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int n_wg = S.nlayers * P.tiles_per_layer;
  hipLaunchKernelGGL(kern, dim3(n_wg), dim3(kBlock), lds, s, P, S);
  return hipGetLastError();
}

template <int KMAX, bool SWEPT>
static hipError_t launch_build_k(const BuildParams &P, const SlabParams &S, bool pack16, bool near,
                                 size_t lds, hipStream_t s)
{
  if constexpr (!SWEPT) {
    if (pack16 && !near && P.paired) return launch_build_t<KMAX, true, false, false, true>(P, S, lds, s);
  }
  if (pack16)
    return near ? launch_build_t<KMAX, true, true, SWEPT>(P, S, lds, s)
                : launch_build_t<KMAX, true, false, SWEPT>(P, S, lds, s);
  return near ? launch_build_t<KMAX, false, true, SWEPT>(P, S, lds, s)
              : launch_build_t<KMAX, false, false, SWEPT>(P, S, lds, s);
}

template <bool SWEPT>
static hipError_t launch_build_sw(const BuildParams &P, const SlabParams &S, int kmax, bool pack16, bool near,
                                  size_t lds, hipStream_t s)
{
  switch (kmax) {
    case 2: return launch_build_k<2, SWEPT>(P, S, pack16, near, lds, s);
    case 4: return launch_build_k<4, SWEPT>(P, S, pack16, near, lds, s);
    case 6: return launch_build_k<6, SWEPT>(P, S, pack16, near, lds, s);
    case 8: return launch_build_k<8, SWEPT>(P, S, pack16, near, lds, s);
    case 10: return launch_build_k<10, SWEPT>(P, S, pack16, near, lds, s);
    case 12: return launch_build_k<12, SWEPT>(P, S, pack16, near, lds, s);
    case 14: return launch_build_k<14, SWEPT>(P, S, pack16, near, lds, s);
    default: return launch_build_k<16, SWEPT>(P, S, pack16, near, lds, s);
  }
}

hipError_t launch_build_slab(const BuildParams &P, const SlabParams &S, int kmax, bool pack16, bool near,
                             bool swept, size_t lds, hipStream_t s)
{
  return swept ? launch_build_sw<true>(P, S, kmax, pack16, near, lds, s)
               : launch_build_sw<false>(P, S, kmax, pack16, near, lds, s);
}

hipError_t launch_batch_build_init(BatchBuildDesc *D, int n, unsigned int *counter,
                                   unsigned long long *pool_top, hipStream_t s)
{
  hipLaunchKernelGGL(k_batch_build_init, dim3((n + 255) / 256), dim3(256), 0, s, D, n, counter, pool_top);
  return hipGetLastError();
}

template <int KMAX, bool NEAR>
static const void *batch_kernel()
{
  return (const void *)k_build_batched<KMAX, NEAR>;
}

static const void *batch_kernel_for(int kmax, bool near)
{
  switch (kmax) {
    case 2: return near ? batch_kernel<2, true>() : batch_kernel<2, false>();
    case 4: return near ? batch_kernel<4, true>() : batch_kernel<4, false>();
    case 6: return near ? batch_kernel<6, true>() : batch_kernel<6, false>();
    case 8: return near ? batch_kernel<8, true>() : batch_kernel<8, false>();
    case 10: return near ? batch_kernel<10, true>() : batch_kernel<10, false>();
    case 12: return near ? batch_kernel<12, true>() : batch_kernel<12, false>();
    case 14: return near ? batch_kernel<14, true>() : batch_kernel<14, false>();
    default: return near ? batch_kernel<16, true>() : batch_kernel<16, false>();
  }
}

hipError_t batch_build_occupancy(int kmax, bool near, size_t lds, int *blocks_per_cu)
{
  const void *k = batch_kernel_for(kmax, near);
  // the persistent kernel also holds a little static LDS (its current item)
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, k);
  if (e != hipSuccess) return e;
  const size_t limit = 160 * 1024 - fa.sharedSizeBytes;
  if (lds > limit) return hipErrorInvalidValue;
  if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)limit)) != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kBlock, lds);
}

hipError_t launch_batch_build(const BatchBuildDesc *D, const BatchItem *items, int n_items, unsigned int *counter,
                              uint64_t *pool, unsigned long long *pool_top, int64_t pool_cap, int kmax, bool near,
                              size_t lds, int grid, hipStream_t s)
{
  void *args[] = {(void *)&D, (void *)&items, (void *)&n_items, (void *)&counter,
                  (void *)&pool, (void *)&pool_top, (void *)&pool_cap};
  return hipLaunchKernel(batch_kernel_for(kmax, near), dim3(grid), dim3(kBlock), args, lds, s);
}

hipError_t launch_batch_scan(BatchBuildDesc *D, int n, hipStream_t s)
{
  hipLaunchKernelGGL(k_batch_scan, dim3(n), dim3(1024), 0, s, D);
  return hipGetLastError();
}

hipError_t launch_batch_copy(const BatchBuildDesc *D, const BatchItem *items, int n_items, const uint64_t *pool,
                             hipStream_t s)
{
  const int grid = n_items < 8192 ? n_items : 8192;
  hipLaunchKernelGGL(k_batch_copy, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, s, D, items, n_items, pool);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(BatchBuildDesc *D, int n, mdp_build_stats *out, hipStream_t s)
{
  hipLaunchKernelGGL(k_batch_finalize, dim3((n + 63) / 64), dim3(64), 0, s, D, n, out);
  return hipGetLastError();
}

hipError_t launch_scan_wg(const SlabParams &S, int n_wg, int64_t *row_ptr_end, hipStream_t s)
{
  hipLaunchKernelGGL(k_scan_wg, dim3(1), dim3(1024), 0, s, S.wg_nnz, n_wg, S.wg_off, S.st, row_ptr_end);
  return hipGetLastError();
}

hipError_t launch_copy(const BuildParams &P, const SlabParams &S, const ModelOut &M, int n_wg, hipStream_t s)
{
  hipLaunchKernelGGL(k_copy, dim3(n_wg), dim3(kBlock), 0, s, P, S, M);
  return hipGetLastError();
}

hipError_t launch_build_finalize(BuildState *st, int64_t capacity, int n_slabs, int near_asked, hipStream_t s)
{
  hipLaunchKernelGGL(k_build_finalize, dim3(1), dim3(64), 0, s, st, capacity, n_slabs, near_asked);
  return hipGetLastError();
}

hipError_t launch_escape_only(const BuildParams &P, BuildState *st, hipStream_t s)
{
  hipLaunchKernelGGL(k_escape_only, dim3(2048), dim3(kBlock), 0, s, P, st);
  return hipGetLastError();
}

hipError_t launch_max_speed(const BuildParams &P, unsigned int *bits, hipStream_t s)
{
  hipLaunchKernelGGL(k_max_speed, dim3(2048), dim3(kBlock), 0, s, P, bits);
  return hipGetLastError();
}

}  // namespace mdpk
