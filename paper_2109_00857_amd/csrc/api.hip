// Host side of the C ABI declared in include/mdp.h: argument checks, launch
// planning (tile shape, realization chunk, LDS size, layers per pass), scratch
// layout, and the enqueue order of the build / value-iteration / policy kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "mdp_internal.h"

using namespace mdpk;

// Launch shape of the build kernel: lanes that own a (cell, action) row (the
// rest of the workgroup helps in the realization phase), realizations per
// chunk, 16- or 32-bit LDS counters.
struct PlanChoice {
  int row_lanes = 0, rch = 0, pack16 = 1;
};

// Shape class of a problem for the tuned-plan table: everything the candidate
// set and the kernel's work balance depend on.
struct TuneKey {
  int na, W, H, kmax, near, nr_log2, nc_log2;
  bool operator==(const TuneKey &o) const
  {
    return na == o.na && W == o.W && H == o.H && kmax == o.kmax && near == o.near && nr_log2 == o.nr_log2 &&
           nc_log2 == o.nc_log2;
  }
};

struct mdp_ctx {
  int device;
  unsigned int *d_small;  // 256 bytes of device memory for synchronous helpers
  void *d_noalloc = nullptr;  // this device's copy of the allocation-free VI scratch
  char noalloc_err[128] = {};
  std::vector<std::pair<TuneKey, PlanChoice>> tuned;  // per shape class, from mdp_autotune / mdp_ctx_set_plan
  char err[512];
  // per-kernel timing (only while profiling is enabled)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[MDP_N_KERNELS];
  size_t ev_used[MDP_N_KERNELS] = {};
};

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kStageBudget = size_t(4) << 30;  // staging bytes per build pass
constexpr int kViGridMaxHost = 8192;  // most workgroups of one sweep launch
constexpr size_t kLdsLimit = 160 * 1024 - 256;  // leaves room for a kernel's static LDS

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void set_err(mdp_ctx *ctx, const char *fmt, ...)
{
  if (!ctx) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
  va_end(ap);
}

int popcount3(uint32_t m) { return (int)(m & 1) + (int)(m >> 1 & 1) + (int)(m >> 2 & 1); }

// Launch plan of one problem (pure host arithmetic).
struct Plan {
  int na, nc, nsg, W;
  bool swept;   // MDP_FLAG_SWEPT_PATH: one more histogram bin (swept-path DEAD)
  int nbins;    // histogram bins: nsg, plus one with the swept-path test
  int max_row;  // most entries of a row: min(nbins, n_real)
  int row_lanes, hw, cells_per_tile, tiles_per_layer, rch;
  bool pack16;
  int kmax;
  size_t lds;
  int layers_per_slab, n_slabs;
  int64_t rows, wg_cap;
  size_t tab_off, stage_off, row_nnz_off, row_off_off, wg_nnz_off, wg_off_off, build_bytes;
  size_t vi_bytes;
};

const char *check_problem(const mdp_problem *p)
{
  if (!p) return "problem is NULL";
  if (p->nx < 1 || p->ny < 1 || p->nt < 1) return "nx, ny, nt must be >= 1";
  if (p->n_modes < 1 || p->n_modes > MDP_MAX_MODES) return "n_modes must be in [1, 16]";
  if (p->n_real < 1 || p->n_real > 65535) return "n_real must be in [1, 65535]";
  if (p->n_head < 1 || p->n_speed < 1 || (int64_t)p->n_head * p->n_speed > MDP_MAX_ACTIONS)
    return "n_head * n_speed must be in [1, 64]";
  if (p->sub_hx < 0 || p->sub_hy < 0) return "sub-grid half widths must be >= 0";
  if (p->target_i < 0 || p->target_i >= p->nx || p->target_j < 0 || p->target_j >= p->ny)
    return "target outside the grid";
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0)) return "dx, dy, dt must be > 0";
  if (!(p->f_max >= 0)) return "f_max must be >= 0";
  if (p->mission_mask == 0 || p->mission_mask > 7u) return "mission_mask must be a nonzero subset of {0,1,2}";
  const int64_t ns = (int64_t)p->nt * p->nx * p->ny;
  if (ns + 2 > INT32_MAX) return "too many states for 32-bit column indices";
  if ((int64_t)p->nx * p->ny > (1 << 24)) return "grid too large";
  return nullptr;
}

// LDS bytes of the build kernel for a launch shape.
size_t plan_lds(int nsg, int na, int row_lanes, int rch, bool pack16)
{
  const size_t fixed_lds = 2 * kMaxA * sizeof(float) + 16 * sizeof(uint32_t);
  const int hw = pack16 ? row_lanes / 2 : row_lanes;
  const int cells = std::min(row_lanes / na, 32);
  return (size_t)nsg * hw * 4 + (size_t)cells * (2 * rch + 4) * 4 + fixed_lds;
}

// Every launch shape the build kernel supports for p (LDS permitting).
std::vector<PlanChoice> plan_candidates(const mdp_problem *p)
{
  std::vector<PlanChoice> out;
  const int na = p->n_head * p->n_speed;
  const int nbins = (2 * p->sub_hx + 1) * (2 * p->sub_hy + 1) + ((p->flags & MDP_FLAG_SWEPT_PATH) ? 1 : 0);
  for (int rl = kBlock; rl >= 64; rl /= 2) {
    if (rl < na) break;
    for (int rch = 64; rch <= 256; rch *= 2)
      for (int pk = 1; pk >= 0; --pk)
        if (plan_lds(nbins, na, rl, rch, pk != 0) <= kLdsLimit) {
          PlanChoice c;
          c.row_lanes = rl;
          c.rch = rch;
          c.pack16 = pk;
          out.push_back(c);
        }
  }
  return out;
}

// Most cell tiles per layer over the candidate shapes (bounds work-list sizes).
int max_tiles_per_layer(const mdp_problem *p)
{
  const int na = std::max(1, p->n_head * p->n_speed);
  const int nc = p->nx * p->ny;
  int cells = 32;
  for (int rl = 64; rl <= kBlock; rl *= 2)
    if (rl >= na) {
      cells = std::min(rl / na, 32);
      break;
    }
  return (nc + std::max(cells, 1) - 1) / std::max(cells, 1);
}

// choice: a launch shape to use (it must fit), or nullptr for the default
// (the widest row mapping that fits, 16-bit counters, chunk from the tile).
const char *make_plan(const mdp_problem *p, Plan &pl, const PlanChoice *choice = nullptr)
{
  if (const char *e = check_problem(p)) return e;
  pl.na = p->n_head * p->n_speed;
  pl.nc = p->nx * p->ny;
  pl.W = 2 * p->sub_hx + 1;
  pl.nsg = pl.W * (2 * p->sub_hy + 1);
  pl.swept = (p->flags & MDP_FLAG_SWEPT_PATH) != 0;
  pl.nbins = pl.nsg + (pl.swept ? 1 : 0);
  pl.max_row = std::min(pl.nbins, p->n_real);
  pl.rows = (int64_t)p->nt * pl.nc * pl.na;
  pl.kmax = mode_bound(p->n_modes);
  bool ok = false;
  if (choice) {
    const int rl = choice->row_lanes;
    if ((rl == 64 || rl == 128 || rl == 256) && rl >= pl.na && (choice->rch == 64 || choice->rch == 128 ||
                                                                 choice->rch == 256)) {
      pl.pack16 = choice->pack16 != 0;
      pl.lds = plan_lds(pl.nbins, pl.na, rl, choice->rch, pl.pack16);
      if (pl.lds <= kLdsLimit) {
        pl.row_lanes = rl;
        pl.hw = pl.pack16 ? rl / 2 : rl;
        pl.cells_per_tile = std::min(rl / pl.na, 32);
        pl.rch = choice->rch;
        ok = true;
      }
    }
    if (!ok) return "launch shape does not fit this problem";
  }
  pl.pack16 = choice ? choice->pack16 != 0 : true;  // n_real <= 65535: two 16-bit counters fit a word
  for (int rl = kBlock; rl >= 64 && !ok; rl /= 2) {
    if (rl < pl.na) break;
    const int cells = std::min(rl / pl.na, 32);
    const int rch = cells <= 8 ? 256 : (cells <= 16 ? 128 : 64);
    const size_t lds = plan_lds(pl.nbins, pl.na, rl, rch, true);
    if (lds <= kLdsLimit) {
      pl.row_lanes = rl;
      pl.hw = rl / 2;
      pl.cells_per_tile = cells;
      pl.rch = rch;
      pl.lds = lds;
      ok = true;
    }
  }
  if (!ok) return "sub-grid too large for the LDS histogram";
  pl.tiles_per_layer = (pl.nc + pl.cells_per_tile - 1) / pl.cells_per_tile;
  pl.wg_cap = (int64_t)pl.cells_per_tile * pl.na * pl.max_row;
  if (pl.wg_cap < 1) pl.wg_cap = 1;
  const size_t rows_per_layer = (size_t)pl.nc * pl.na;
  const size_t per_layer = (size_t)pl.tiles_per_layer * pl.wg_cap * 8;
  int L = (int)std::max<size_t>(1, kStageBudget / std::max<size_t>(per_layer, 1));
  L = std::min(L, p->nt);
  pl.layers_per_slab = L;
  pl.n_slabs = (p->nt + L - 1) / L;
  const size_t slab_rows = rows_per_layer * L;
  const size_t slab_wgs = (size_t)pl.tiles_per_layer * L;
  size_t off = align_up(sizeof(BuildState));
  pl.tab_off = off;
  off = align_up(off + 2 * kMaxA * sizeof(float));
  pl.row_nnz_off = off;
  off = align_up(off + slab_rows * 4);
  pl.row_off_off = off;
  off = align_up(off + slab_rows * 4);
  pl.wg_nnz_off = off;
  off = align_up(off + slab_wgs * 4);
  pl.wg_off_off = off;
  off = align_up(off + slab_wgs * 8);
  pl.stage_off = off;
  off = align_up(off + slab_wgs * (size_t)pl.wg_cap * 8);
  pl.build_bytes = off;
  const int64_t ns = (int64_t)p->nt * pl.nc;
  pl.vi_bytes = align_up(sizeof(VIState)) + align_up(sizeof(mdp_vi_stats)) + align_up((size_t)ns * 8) +
                align_up(sizeof(double) * kViGridMaxHost);
  return nullptr;
}

TuneKey tune_key(const mdp_problem *p)
{
  auto lg = [](int64_t x) {
    int k = 0;
    while ((int64_t)1 << k < x) ++k;
    return k;
  };
  TuneKey k;
  k.na = p->n_head * p->n_speed;
  k.W = 2 * p->sub_hx + 1;
  k.H = 2 * p->sub_hy + 1;
  k.kmax = mode_bound(p->n_modes);
  k.near = (p->flags & MDP_FLAG_NEAR_EDGE) ? 1 : 0;
  k.nr_log2 = lg(p->n_real);
  k.nc_log2 = lg((int64_t)p->nx * p->ny);
  return k;
}

// The tuned launch shape of p's class on this context, or nullptr.
const PlanChoice *tuned_choice(const mdp_ctx *ctx, const mdp_problem *p)
{
  if (!ctx || !p) return nullptr;
  const TuneKey k = tune_key(p);
  for (const auto &e : ctx->tuned)
    if (e.first == k) return &e.second;
  return nullptr;
}

// Plan of p on ctx: its tuned shape when it fits, else the default.
const char *ctx_plan(const mdp_ctx *ctx, const mdp_problem *p, Plan &pl)
{
  if (const PlanChoice *c = tuned_choice(ctx, p))
    if (!make_plan(p, pl, c)) return nullptr;
  return make_plan(p, pl);
}

bool is_device_ptr(const void *ptr)
{
  if (!ptr) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Displacement tables in cell units, evaluated in double and rounded once.
// Headings along an axis (whole quarter turns) take the exact direction
// (1, 0), (0, 1), (-1, 0) or (0, -1).
void action_tables(const mdp_problem *p, float *hx, float *hy)
{
  const double kPi = 3.14159265358979323846;
  static const double kAxis[4][2] = {{1.0, 0.0}, {0.0, 1.0}, {-1.0, 0.0}, {0.0, -1.0}};
  for (int jf = 0; jf < p->n_speed; ++jf) {
    const double F = p->f_max * (double)(jf + 1) / (double)p->n_speed;
    for (int h = 0; h < p->n_head; ++h) {
      const double th = 2.0 * kPi * (double)h / (double)p->n_head;
      const bool axis = (4 * h) % p->n_head == 0;
      const double dirx = axis ? kAxis[4 * h / p->n_head][0] : cos(th);
      const double diry = axis ? kAxis[4 * h / p->n_head][1] : sin(th);
      const int a = jf * p->n_head + h;
      hx[a] = (float)(F * dirx * p->dt / p->dx);
      hy[a] = (float)(F * diry * p->dt / p->dy);
    }
  }
}

// Largest |flow speed| that cannot push any landing out of the sub-grid.
// |px - (i + 1/2)| <= |u| dt/dx + ulp terms; X adds at most max|H| and one more
// rounding; both roundings are bounded by 4 ulp of the largest coordinate.
float safe_speed(int h, double hmax_abs, double lam, int n)
{
  const double coord = (double)n + h + 2.0;
  const double ulp = ldexp(1.0, (int)ceil(log2(coord)) - 23);
  const double margin = 4.0 * ulp + 1e-6;
  const double s = ((double)h + 0.5 - hmax_abs - margin) / lam;
  if (s <= 0) return -1.0f;
  float f = (float)s;
  if ((double)f > s) f = nextafterf(f, 0.0f);
  return f;
}

// Pairs of actions for the paired landing loop: actions with bitwise-equal Hx
// first (headings h and N_h - h, where the rounded tables agree, and the axis
// headings N_h/4 and 3N_h/4, whose Hx are exact zeros; the x add,
// floor and column offset of a landing then serve both rows), the remaining
// actions paired in ascending order. Off (paired = 0) for an odd N_a or when
// no two actions share Hx.
static void pair_actions(int na, const float *hx, BuildParams &P)
{
  P.paired = 0;
  P.n_real_pairs = 0;
  if (na < 2 || (na & 1)) return;
  bool used[kMaxA] = {};
  int q = 0;
  for (int a = 0; a < na; ++a) {
    if (used[a]) continue;
    for (int b = a + 1; b < na; ++b)
      if (!used[b] && memcmp(&hx[a], &hx[b], sizeof(float)) == 0) {
        used[a] = used[b] = true;
        P.pair_a[2 * q] = (uint8_t)a;
        P.pair_a[2 * q + 1] = (uint8_t)b;
        ++q;
        break;
      }
  }
  P.n_real_pairs = q;
  int pending = -1;
  for (int a = 0; a < na; ++a) {
    if (used[a]) continue;
    if (pending < 0) {
      pending = a;
    } else {
      P.pair_a[2 * q] = (uint8_t)pending;
      P.pair_a[2 * q + 1] = (uint8_t)a;
      ++q;
      pending = -1;
    }
  }
  for (int k = 0; k < 2 * q; ++k) P.row_pair[P.pair_a[k]] = (uint8_t)((k >> 1) << 1 | (k & 1));
  P.paired = P.n_real_pairs > 0 ? 1 : 0;
}

void fill_params(const mdp_problem *p, const mdp_env *env, const mdp_model *model, const Plan &pl,
                 BuildParams &P, ActionTables &T)
{
  memset(&P, 0, sizeof(P));
  P.ubar = env->ubar;
  P.vbar = env->vbar;
  P.phiu = env->phiu;
  P.phiv = env->phiv;
  P.mu = env->mu;
  P.gbar = env->gbar;
  P.mask = env->mask;
  P.reward = model ? model->reward : nullptr;
  P.rows = pl.rows;
  P.nx = p->nx;
  P.ny = p->ny;
  P.nt = p->nt;
  P.nc = pl.nc;
  P.na = pl.na;
  P.nr = p->n_real;
  P.K = p->n_modes;
  P.hx = p->sub_hx;
  P.hy = p->sub_hy;
  P.W = pl.W;
  P.nsg = pl.nsg;
  P.nbins = pl.nbins;
  P.ti = p->target_i;
  P.tj = p->target_j;
  P.mean_tstride = p->mean_time_varying ? pl.nc : 0;
  P.mode_tstride = p->mode_time_varying ? (int64_t)p->n_modes * pl.nc : 0;
  P.cells_per_tile = pl.cells_per_tile;
  P.tiles_per_layer = pl.tiles_per_layer;
  P.rch = pl.rch;
  P.row_lanes = pl.row_lanes;
  P.hw = pl.hw;
  P.nmiss = 0;
  for (int m = 0; m < 3; ++m)
    if (p->mission_mask >> m & 1u) P.miss[P.nmiss++] = m;
  P.n_head = p->n_head;
  P.n_speed = p->n_speed;
  P.lam_x = (float)(p->dt / p->dx);
  P.lam_y = (float)(p->dt / p->dy);
  P.eps_x = (float)(1e-6 / p->dx);
  P.eps_y = (float)(1e-6 / p->dy);
  P.dt = p->dt;
  P.r_term = p->r_term;
  P.r_out = p->r_outbound;
  P.c_f = p->c_f;
  P.c_r = p->c_r;
  P.f_max = p->f_max;
  memset(&T, 0, sizeof(T));
  action_tables(p, T.hx, T.hy);
  double mx = 0.0, my = 0.0;
  for (int a = 0; a < pl.na; ++a) {
    mx = std::max(mx, fabs((double)T.hx[a]));
    my = std::max(my, fabs((double)T.hy[a]));
  }
  P.usafe = safe_speed(p->sub_hx, mx, p->dt / p->dx, p->nx);
  P.vsafe = safe_speed(p->sub_hy, my, p->dt / p->dy, p->ny);
  pair_actions(pl.na, T.hx, P);
}

// Events bracketing one launch of kernel kind k (no-ops unless profiling).
struct Timed {
  mdp_ctx *ctx;
  int k;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  Timed(mdp_ctx *c, int kind, hipStream_t st) : ctx(c), k(kind), s(st)
  {
    if (!ctx || !ctx->profiling) return;
    auto &v = ctx->ev[k];
    if (ctx->ev_used[k] == v.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      v.emplace_back(a, b);
    }
    auto &pr = v[ctx->ev_used[k]++];
    (void)hipEventRecord(pr.first, s);
    stop = pr.second;
  }
  ~Timed()
  {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

mdp_status hip_fail(mdp_ctx *ctx, hipError_t e, const char *where)
{
  set_err(ctx, "%s: %s", where, hipGetErrorString(e));
  return MDP_E_HIP;
}

}  // namespace

extern "C" {

const char *mdp_status_str(mdp_status s)
{
  switch (s) {
    case MDP_OK: return "ok";
    case MDP_E_INVALID: return "invalid argument";
    case MDP_E_CAPACITY: return "nnz capacity too small";
    case MDP_E_SUBGRID: return "landing outside the neighbouring sub-grid";
    case MDP_E_HIP: return "HIP runtime error";
    case MDP_E_NOT_CONVERGED: return "value iteration did not converge";
    case MDP_E_SCRATCH: return "scratch buffer too small";
    default: return "unknown status";
  }
}

mdp_status mdp_ctx_create(int32_t device, mdp_ctx **out)
{
  if (!out) return MDP_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MDP_E_INVALID;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return MDP_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return MDP_E_HIP;
  mdp_ctx *ctx = new mdp_ctx();
  ctx->device = device;
  ctx->err[0] = 0;
  hipError_t e = hipMalloc((void **)&ctx->d_small, 256);
  if (e == hipSuccess) {  // with `device` current: the device's copy of the static scratch
    const hipError_t es = noalloc_scratch(device, &ctx->d_noalloc);
    if (es != hipSuccess) {
      ctx->d_noalloc = nullptr;
      snprintf(ctx->noalloc_err, sizeof(ctx->noalloc_err), "%s", hipGetErrorString(es));
    }
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    delete ctx;
    return MDP_E_HIP;
  }
  *out = ctx;
  return MDP_OK;
}

mdp_status mdp_ctx_destroy(mdp_ctx *ctx)
{
  if (!ctx) return MDP_E_INVALID;
  if (ctx->d_small) (void)hipFree(ctx->d_small);
  for (auto &v : ctx->ev)
    for (auto &pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  delete ctx;
  return MDP_OK;
}

const char *mdp_last_error(const mdp_ctx *ctx) { return ctx ? ctx->err : ""; }

mdp_status mdp_ctx_profile(mdp_ctx *ctx, int32_t enable)
{
  if (!ctx) return MDP_E_INVALID;
  if (enable)
    for (size_t &u : ctx->ev_used) u = 0;
  ctx->profiling = enable != 0;
  return MDP_OK;
}

mdp_status mdp_ctx_profile_read(mdp_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms)
{
  if (!ctx || kernel < 0 || kernel >= MDP_N_KERNELS || !launches || !total_ms) return MDP_E_INVALID;
  double tot = 0.0;
  for (size_t i = 0; i < ctx->ev_used[kernel]; ++i) {
    auto &pr = ctx->ev[kernel][i];
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(ctx, e, "event sync");
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, pr.first, pr.second)) != hipSuccess) return hip_fail(ctx, e, "elapsed");
    tot += ms;
  }
  *launches = (int64_t)ctx->ev_used[kernel];
  *total_ms = tot;
  return MDP_OK;
}

mdp_status mdp_build_query(const mdp_problem *p, mdp_sizes *out)
{
  if (!out) return MDP_E_INVALID;
  Plan pl;
  if (make_plan(p, pl)) return MDP_E_INVALID;
  memset(out, 0, sizeof(*out));
  out->n_states = (int64_t)p->nt * pl.nc;
  out->n_actions = pl.na;
  out->n_rows = pl.rows;
  out->n_sg = pl.nsg;
  out->nnz_upper = pl.rows * (int64_t)pl.max_row;
  out->n_missions = popcount3(p->mission_mask);
  size_t build_bytes = pl.build_bytes;  // enough for any launch shape a context may use
  for (const PlanChoice &c : plan_candidates(p)) {
    Plan q;
    if (!make_plan(p, q, &c)) build_bytes = std::max(build_bytes, q.build_bytes);
  }
  out->scratch_bytes = (int64_t)std::max(build_bytes, pl.vi_bytes);
  const int64_t tm = p->mean_time_varying ? p->nt : 1, tp = p->mode_time_varying ? p->nt : 1;
  out->env_bytes = 4 * (2 * tm * pl.nc + 2 * tp * (int64_t)p->n_modes * pl.nc +
                        (int64_t)p->nt * p->n_modes * p->n_real) +
                   (int64_t)(p->nt + 1) * pl.nc * 5;
  out->layers_per_slab = pl.layers_per_slab;
  return MDP_OK;
}

static const char *check_env(const mdp_problem *p, const mdp_env *env)
{
  if (!env) return "env is NULL";
  if (!is_device_ptr(env->ubar) || !is_device_ptr(env->vbar)) return "ubar/vbar must be device pointers";
  if (!is_device_ptr(env->phiu) || !is_device_ptr(env->phiv)) return "phiu/phiv must be device pointers";
  if (!is_device_ptr(env->mu)) return "mu must be a device pointer";
  if ((p->mission_mask >> MDP_MISSION_NET_ENERGY & 1u) && !is_device_ptr(env->gbar))
    return "the net-energy mission needs gbar on the device";
  if (env->gbar && !is_device_ptr(env->gbar)) return "gbar must be a device pointer";
  if (env->mask && !is_device_ptr(env->mask)) return "mask must be a device pointer";
  return nullptr;
}

mdp_status mdp_subgrid_auto(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, int32_t *hx,
                            int32_t *hy, void *stream)
{
  if (!ctx || !hx || !hy) return MDP_E_INVALID;
  mdp_problem q = *p;
  q.sub_hx = q.sub_hy = 0;
  Plan pl;
  if (const char *e = make_plan(&q, pl)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (const char *e = check_env(&q, env)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  BuildParams P;
  ActionTables T;
  fill_params(&q, env, nullptr, pl, P, T);
  hipError_t e = hipMemsetAsync(ctx->d_small, 0, 8, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "memset");
  if ((e = launch_max_speed(P, ctx->d_small, s)) != hipSuccess) return hip_fail(ctx, e, "max_speed");
  unsigned int bits[2];
  if ((e = hipMemcpyAsync(bits, ctx->d_small, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(ctx, e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(ctx, e, "sync");
  float U, V;
  memcpy(&U, &bits[0], 4);
  memcpy(&V, &bits[1], 4);
  auto half = [](double S, double fmax, double lam) {
    const double z = (S + fmax) * lam + 1e-3;
    const int32_t h = (int32_t)floor(z - 0.5) + 1;
    return h < 0 ? 0 : h;
  };
  *hx = half((double)U, p->f_max, p->dt / p->dx);
  *hy = half((double)V, p->f_max, p->dt / p->dy);
  return MDP_OK;
}

static mdp_status build_with_plan(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                                  void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream,
                                  const Plan &pl, int t_begin = 0);
static void fill_vi_params(const mdp_problem *p, const mdp_model *model, const Plan &pl, int mission, int n_wg,
                           VIParams &V);

mdp_status mdp_build(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                     void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream)
{
  if (!ctx) return MDP_E_INVALID;
  Plan pl;
  if (const char *e = ctx_plan(ctx, p, pl)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  return build_with_plan(ctx, p, env, model, scratch, scratch_bytes, stats, stream, pl);
}

mdp_status mdp_build_from(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                          int32_t t0, void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream)
{
  if (!ctx) return MDP_E_INVALID;
  Plan pl;
  if (const char *e = ctx_plan(ctx, p, pl)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (t0 < 0 || t0 >= p->nt) {
    set_err(ctx, "t0 must be in [0, nt)");
    return MDP_E_INVALID;
  }
  return build_with_plan(ctx, p, env, model, scratch, scratch_bytes, stats, stream, pl, t0);
}

// Build of the layers [t_begin, nt) (all of them for mdp_build). With
// t_begin > 0 the entries of the earlier layers stay where they are and the
// rebuilt layers' entries follow them (the running count starts at the row
// pointer of layer t_begin's first row).
static mdp_status build_with_plan(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                                  void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream,
                                  const Plan &pl, int t_begin)
{
  if (const char *e = check_env(p, env)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (!model || !is_device_ptr(model->row_ptr) || !is_device_ptr(model->reward) ||
      (model->nnz_capacity > 0 && (!is_device_ptr(model->col) || !is_device_ptr(model->cnt))) ||
      (model->ent && !is_device_ptr(model->ent)) || (model->roff && !is_device_ptr(model->roff))) {
    set_err(ctx, "model buffers must be device pointers");
    return MDP_E_INVALID;
  }
  if ((model->ent == nullptr) != (model->roff == nullptr)) {
    set_err(ctx, "ent and roff go together");
    return MDP_E_INVALID;
  }
  if (!stats) {
    set_err(ctx, "stats is NULL");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(scratch) || scratch_bytes < pl.build_bytes) {
    set_err(ctx, "scratch needs %zu device bytes", pl.build_bytes);
    return MDP_E_SCRATCH;
  }
  hipStream_t s = (hipStream_t)stream;
  BuildParams P;
  ActionTables T;
  fill_params(p, env, model, pl, P, T);
  char *sc = (char *)scratch;
  BuildState *st = (BuildState *)sc;
  P.tab = (const float *)(sc + pl.tab_off);
  hipError_t e;
  if ((e = t_begin > 0 ? launch_build_init_from(st, model->row_ptr + (int64_t)t_begin * pl.nc * pl.na, s)
                       : launch_build_init(st, s)) != hipSuccess)
    return hip_fail(ctx, e, "init");
  if ((e = launch_fill_tab(T, (float *)(sc + pl.tab_off), s)) != hipSuccess) return hip_fail(ctx, e, "tables");
  const bool near = (p->flags & MDP_FLAG_NEAR_EDGE) != 0;
  // A sub-grid that cannot hold the agent's own displacement cannot be
  // histogrammed safely: count the escapes exactly and stop there.
  double mx = 0.0, my = 0.0;
  for (int a = 0; a < pl.na; ++a) {
    mx = std::max(mx, fabs((double)T.hx[a]));
    my = std::max(my, fabs((double)T.hy[a]));
  }
  const bool tiny = (safe_speed(p->sub_hx, mx, 1.0, p->nx) < 0.0f) || (safe_speed(p->sub_hy, my, 1.0, p->ny) < 0.0f);
  int n_slabs = 0;
  if (tiny) {
    if ((e = launch_escape_only(P, st, s)) != hipSuccess) return hip_fail(ctx, e, "escape_only");
  } else {
    ModelOut M{model->row_ptr, model->col, model->cnt, model->nnz_capacity};
    for (int t0 = t_begin; t0 < p->nt; t0 += pl.layers_per_slab, ++n_slabs) {
      SlabParams S;
      S.t0 = t0;
      S.nlayers = std::min(pl.layers_per_slab, p->nt - t0);
      S.row0 = (int64_t)t0 * pl.nc * pl.na;
      S.row_nnz = (uint32_t *)(sc + pl.row_nnz_off);
      S.row_off = (uint32_t *)(sc + pl.row_off_off);
      S.wg_nnz = (uint32_t *)(sc + pl.wg_nnz_off);
      S.wg_off = (int64_t *)(sc + pl.wg_off_off);
      S.stage = (uint64_t *)(sc + pl.stage_off);
      S.wg_cap = pl.wg_cap;
      S.st = st;
      const int n_wg = S.nlayers * pl.tiles_per_layer;
      {
        Timed tm(ctx, MDP_KERNEL_BUILD, s);
        if ((e = launch_build_slab(P, S, pl.kmax, pl.pack16, near, pl.swept, pl.lds, s)) != hipSuccess)
          return hip_fail(ctx, e, "build");
      }
      const bool last = t0 + S.nlayers >= p->nt;
      if ((e = launch_scan_wg(S, n_wg, last ? model->row_ptr + pl.rows : nullptr, s)) != hipSuccess)
        return hip_fail(ctx, e, "scan");
      {
        Timed tm(ctx, MDP_KERNEL_COPY, s);
        if ((e = launch_copy(P, S, M, n_wg, s)) != hipSuccess) return hip_fail(ctx, e, "copy");
      }
    }
  }
  if (!tiny && model->ent) {  // the fused sweep's packed entries of the rebuilt layers
    int mission = 0;
    while (!(p->mission_mask >> mission & 1u)) ++mission;
    VIParams V;
    fill_vi_params(p, model, pl, mission, kViGridMaxHost, V);
    if (V.ent) {
      Timed tm(ctx, MDP_KERNEL_COPY, s);
      if ((e = launch_compact(V, model->ent, model->roff, t_begin, s)) != hipSuccess) return hip_fail(ctx, e, "pack");
    }
  }
  if ((e = launch_build_finalize(st, model->nnz_capacity, n_slabs, near ? 1 : 0, s)) != hipSuccess)
    return hip_fail(ctx, e, "finalize");
  if ((e = hipMemcpyAsync(stats, &st->out, sizeof(mdp_build_stats), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(ctx, e, "stats copy");
  return MDP_OK;
}

mdp_status mdp_build_sync(mdp_ctx *ctx, const mdp_build_stats *stats, void *stream)
{
  if (!ctx || !stats) return MDP_E_INVALID;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "build sync");
  switch (stats->status) {
    case MDP_OK: return MDP_OK;
    case MDP_E_CAPACITY:
      set_err(ctx, "the model needs %lld nonzeros", (long long)stats->nnz);
      return MDP_E_CAPACITY;
    case MDP_E_SUBGRID:
      set_err(ctx, "%lld landings left the sub-grid", (long long)stats->n_escape);
      return MDP_E_SUBGRID;
    default:
      set_err(ctx, "build reported status %d", (int)stats->status);
      return stats->status;
  }
}

// Sweep parameters of mission `mission` of a built model.
static void fill_vi_params(const mdp_problem *p, const mdp_model *model, const Plan &pl, int mission, int n_wg,
                           VIParams &V)
{
  int slot = 0;
  for (int m = 0; m < mission; ++m) slot += (int)(p->mission_mask >> m & 1u);
  memset(&V, 0, sizeof(V));
  V.row_ptr = model->row_ptr;
  V.col = model->col;
  V.cnt = model->cnt;
  V.R = model->reward + (int64_t)slot * pl.rows;
  V.cap = model->nnz_capacity;
  V.ns = (int64_t)p->nt * pl.nc;
  V.na = pl.na;
  V.nx = p->nx;
  V.ny = p->ny;
  V.nc = pl.nc;
  V.nt = p->nt;
  V.hy = p->sub_hy;
  V.hx = p->sub_hx;
  V.states_per_wg = std::min(kViRows / pl.na, pl.nc);
  V.blocks_per_layer = (pl.nc + V.states_per_wg - 1) / V.states_per_wg;
  V.n_blocks = (int64_t)p->nt * V.blocks_per_layer;
  V.win_rows = vi_window_rows(p->nx, p->ny, p->sub_hy, V.states_per_wg);
  V.narrow = 4 * (V.states_per_wg + 2 * p->sub_hx) <= p->nx ? 1 : 0;
  // packed entries exist only with the window, and with every block's entries
  // addressable by 16-bit row offsets
  const bool offs16 = (int64_t)V.states_per_wg * pl.na * pl.max_row <= 0xFFFF;
  V.ent = (V.win_rows > 0 && offs16) ? model->ent : nullptr;
  V.roff = V.ent ? model->roff : nullptr;
  V.max_row = pl.max_row;
  V.n_wg = n_wg;
  V.inv_nr = 1.0 / (double)p->n_real;
}

// ---------------------------------------------------------------- autotuning
// The sample a launch shape is timed on: the problem's first layers, enough
// of them for kTuneTiles cell tiles of the default shape (many waves of
// resident workgroups, so the timing is the steady state, not the tail).
static constexpr double kTuneTiles = 32768;
static constexpr int kTuneRounds = 4;  // timed rounds over all candidates

static const char *tune_sample(const mdp_problem *p, mdp_problem &q)
{
  Plan pl;
  if (const char *e = make_plan(p, pl)) return e;
  q = *p;
  q.nt = (int32_t)std::max(1.0, std::min((double)p->nt, std::ceil(kTuneTiles / std::max(pl.tiles_per_layer, 1))));
  return nullptr;
}

struct TuneLayout {
  size_t row_ptr, col, cnt, reward, scratch, total, build_bytes;
  int64_t rows, cap;
};

static const char *tune_layout(const mdp_problem *q, TuneLayout &T)
{
  Plan pl;
  if (const char *e = make_plan(q, pl)) return e;
  T.rows = pl.rows;
  T.cap = pl.rows * (int64_t)pl.max_row;
  T.build_bytes = pl.build_bytes;
  for (const PlanChoice &c : plan_candidates(q)) {
    Plan x;
    if (!make_plan(q, x, &c)) T.build_bytes = std::max(T.build_bytes, x.build_bytes);
  }
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = align_up(off + b);
    return at;
  };
  T.row_ptr = take(8 * (size_t)(T.rows + 1));
  T.col = take(4 * (size_t)T.cap);
  T.cnt = take(2 * (size_t)T.cap);
  T.reward = take(4 * (size_t)T.rows * popcount3(q->mission_mask));
  T.scratch = take(T.build_bytes);
  T.total = off;
  return nullptr;
}

mdp_status mdp_autotune_query(const mdp_problem *p, size_t *scratch_bytes)
{
  if (!scratch_bytes) return MDP_E_INVALID;
  mdp_problem q;
  TuneLayout T;
  if (tune_sample(p, q) || tune_layout(&q, T)) return MDP_E_INVALID;
  *scratch_bytes = T.total;
  return MDP_OK;
}

mdp_status mdp_autotune(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, void *scratch, size_t scratch_bytes,
                        mdp_tune_report *out, void *stream)
{
  if (!ctx || !out) return MDP_E_INVALID;
  mdp_problem q;
  TuneLayout T;
  if (const char *e = tune_sample(p, q)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (const char *e = tune_layout(&q, T)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(scratch) || scratch_bytes < T.total) {
    set_err(ctx, "autotune scratch needs %zu device bytes", T.total);
    return MDP_E_SCRATCH;
  }
  const std::vector<PlanChoice> cands = plan_candidates(&q);
  if (cands.empty() || (int)cands.size() > MDP_MAX_TUNE) {
    set_err(ctx, "no launch shape fits this problem");
    return MDP_E_INVALID;
  }
  char *sc = (char *)scratch;
  mdp_model M{(int64_t *)(sc + T.row_ptr), (int32_t *)(sc + T.col), (uint16_t *)(sc + T.cnt),
              (float *)(sc + T.reward), T.cap};
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(ctx, e, "autotune events");
  }
  memset(out, 0, sizeof(*out));
  out->sample_layers = q.nt;
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  mdp_status rc = MDP_OK;
  // Round robin over the candidates, kTuneRounds times after one warm-up
  // round; each keeps its fastest time (drift of clocks over the sweep hits
  // every candidate alike).
  std::vector<Plan> plans(cands.size());
  std::vector<double> ms_best(cands.size(), 1e30);
  for (size_t i = 0; i < cands.size(); ++i) make_plan(&q, plans[i], &cands[i]);
  for (int round = 0; round <= kTuneRounds && rc == MDP_OK; ++round) {
    for (size_t i = 0; i < cands.size() && rc == MDP_OK; ++i) {
      mdp_build_stats st;
      if ((e = hipEventRecord(e0, s)) != hipSuccess) rc = hip_fail(ctx, e, "autotune record");
      if (rc == MDP_OK) rc = build_with_plan(ctx, &q, env, &M, sc + T.scratch, T.build_bytes, &st, stream, plans[i]);
      if (rc == MDP_OK && (e = hipEventRecord(e1, s)) != hipSuccess) rc = hip_fail(ctx, e, "autotune record");
      if (rc == MDP_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(ctx, e, "autotune sync");
      float ms = 0.0f;
      if (rc == MDP_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_fail(ctx, e, "elapsed");
      if (rc == MDP_OK && st.status != MDP_OK) {
        set_err(ctx, "autotune sample build failed: %s", mdp_status_str(st.status));
        rc = st.status;
      }
      if (rc == MDP_OK && round > 0) ms_best[i] = std::min(ms_best[i], (double)ms);
    }
  }
  int best = -1;
  for (size_t i = 0; i < cands.size(); ++i) {
    out->row_lanes[i] = cands[i].row_lanes;
    out->rch[i] = cands[i].rch;
    out->pack16[i] = cands[i].pack16;
    out->ms[i] = ms_best[i];
    if (best < 0 || ms_best[i] < out->ms[best]) best = (int)i;
  }
  ctx->profiling = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MDP_OK) return rc;
  out->n_candidates = (int32_t)cands.size();
  out->best = best;
  out->default_shape = -1;
  Plan dpl;
  if (!make_plan(&q, dpl))
    for (size_t i = 0; i < cands.size(); ++i)
      if (cands[i].row_lanes == dpl.row_lanes && cands[i].rch == dpl.rch && (cands[i].pack16 != 0) == dpl.pack16)
        out->default_shape = (int32_t)i;
  return mdp_ctx_set_plan(ctx, p, cands[best].row_lanes, cands[best].rch, cands[best].pack16);
}

mdp_status mdp_ctx_set_plan(mdp_ctx *ctx, const mdp_problem *p, int32_t row_lanes, int32_t rch, int32_t pack16)
{
  if (!ctx || !p) return MDP_E_INVALID;
  const TuneKey k = tune_key(p);
  for (size_t i = 0; i < ctx->tuned.size(); ++i)
    if (ctx->tuned[i].first == k) {
      ctx->tuned.erase(ctx->tuned.begin() + (long)i);
      break;
    }
  if (row_lanes == 0) return MDP_OK;  // back to the default shape
  PlanChoice c;
  c.row_lanes = row_lanes;
  c.rch = rch;
  c.pack16 = pack16 ? 1 : 0;
  Plan pl;
  if (const char *e = make_plan(p, pl, &c)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  ctx->tuned.push_back({k, c});
  return MDP_OK;
}

static mdp_status vi_setup(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                           Plan &pl, VIParams &V)
{
  if (!ctx) return MDP_E_INVALID;
  if (const char *e = make_plan(p, pl)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (mission < 0 || mission > 2 || !(p->mission_mask >> mission & 1u)) {
    set_err(ctx, "mission %d was not built", mission);
    return MDP_E_INVALID;
  }
  if (!model || !is_device_ptr(model->row_ptr) || !is_device_ptr(model->col) || !is_device_ptr(model->cnt) ||
      !is_device_ptr(model->reward) || (model->ent && !is_device_ptr(model->ent)) ||
      (model->roff && !is_device_ptr(model->roff))) {
    set_err(ctx, "model buffers must be device pointers");
    return MDP_E_INVALID;
  }
  if ((model->ent == nullptr) != (model->roff == nullptr)) {
    set_err(ctx, "ent and roff go together");
    return MDP_E_INVALID;
  }
  fill_vi_params(p, model, pl, mission, kViGridMaxHost, V);
  return MDP_OK;
}

}  // extern "C"

// Sweeps of one mission over layers [t_first, nt) from the values in d_v, on
// the value-iteration scratch at sc (at least pl.vi_bytes: sweep state, device
// stats, second value buffer, per-workgroup residuals), then the stats copy.
// `timed`: record the sweeps in the context's profile.
static mdp_status vi_run(mdp_ctx *ctx, const mdp_problem *p, VIParams &V, int t_first, double tol,
                         int32_t max_sweeps, double *d_v, char *sc, mdp_vi_stats *stats, void *stream, bool timed)
{
  V.st = (VIState *)sc;
  V.t_lo = t_first;
  mdp_vi_stats *dstats = (mdp_vi_stats *)(sc + align_up(sizeof(VIState)));
  double *v_alt = (double *)(sc + align_up(sizeof(VIState)) + align_up(sizeof(mdp_vi_stats)));
  double *wg_res = (double *)((char *)v_alt + align_up((size_t)V.ns * 8));
  V.tol = tol;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = launch_vi_init(V.st, 1, s)) != hipSuccess) return hip_fail(ctx, e, "vi init");
  // The model is layered in time, so a positive tolerance is met after at most
  // nt - t_first + 1 sweeps (the last one has residual exactly 0): no host
  // polling.
  int n = max_sweeps;
  if (tol > 0.0) n = std::min(n, p->nt - t_first + 1);
  for (int k = 0; k < n; ++k) {
    const double *vin = (k & 1) ? v_alt : d_v;
    double *vout = (k & 1) ? d_v : v_alt;
    Timed tm(timed ? ctx : nullptr, MDP_KERNEL_VI_SWEEP, s);
    if ((e = launch_vi_sweep(V, vin, vout, vi_active_layers(p->nt, k), wg_res, s)) != hipSuccess)
      return hip_fail(ctx, e, "vi sweep");
  }
  if ((e = launch_vi_finish(V, d_v, v_alt, dstats, s)) != hipSuccess) return hip_fail(ctx, e, "vi finish");
  if ((e = hipMemcpyAsync(stats, dstats, sizeof(mdp_vi_stats), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(ctx, e, "vi stats copy");
  return MDP_OK;
}

extern "C" {

mdp_status mdp_value_iterate(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                             double tol, int32_t max_sweeps, double *d_v, void *scratch, size_t scratch_bytes,
                             mdp_vi_stats *stats, void *stream)
{
  return mdp_value_iterate_layers(ctx, p, model, mission, 0, tol, max_sweeps, d_v, scratch, scratch_bytes, stats,
                                  stream);
}

mdp_status mdp_value_iterate_layers(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                                    int32_t t_first, double tol, int32_t max_sweeps, double *d_v, void *scratch,
                                    size_t scratch_bytes, mdp_vi_stats *stats, void *stream)
{
  Plan pl;
  VIParams V;
  mdp_status rc = vi_setup(ctx, p, model, mission, pl, V);
  if (rc != MDP_OK) return rc;
  if (t_first < 0 || t_first >= p->nt) {
    set_err(ctx, "t_first must be in [0, nt)");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(d_v) || !stats || max_sweeps < 0) {
    set_err(ctx, "d_v must be a device pointer, stats non-NULL, max_sweeps >= 0");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(scratch) || scratch_bytes < pl.vi_bytes) {
    set_err(ctx, "scratch needs %zu device bytes", pl.vi_bytes);
    return MDP_E_SCRATCH;
  }
  return vi_run(ctx, p, V, t_first, tol, max_sweeps, d_v, (char *)scratch, stats, stream, true);
}

mdp_status mdp_value_iterate_noalloc(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                                     double tol, int32_t max_sweeps, double *d_v, mdp_vi_stats *stats, void *stream)
{
  Plan pl;
  VIParams V;
  mdp_status rc = vi_setup(ctx, p, model, mission, pl, V);
  if (rc != MDP_OK) return rc;
  if (pl.vi_bytes > MDP_NOALLOC_SCRATCH_BYTES) {
    set_err(ctx, "value iteration of %lld states needs %zu scratch bytes, above the %zu of the allocation-free path",
            (long long)V.ns, pl.vi_bytes, (size_t)MDP_NOALLOC_SCRATCH_BYTES);
    return MDP_E_SCRATCH;
  }
  if (!is_device_ptr(d_v) || !stats || max_sweeps < 0) {
    set_err(ctx, "d_v must be a device pointer, stats non-NULL, max_sweeps >= 0");
    return MDP_E_INVALID;
  }
  if (!ctx->d_noalloc) {
    set_err(ctx, "the allocation-free scratch of device %d was not set up: %s", ctx->device, ctx->noalloc_err);
    return MDP_E_HIP;
  }
  return vi_run(ctx, p, V, 0, tol, max_sweeps, d_v, (char *)ctx->d_noalloc, stats, stream, false);
}

mdp_status mdp_value_iterate_missions(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model,
                                      int32_t n_missions, const int32_t *missions, double tol, int32_t max_sweeps,
                                      double *const *d_v, void *scratch, size_t scratch_bytes, mdp_vi_stats *stats,
                                      void *stream)
{
  if (!ctx) return MDP_E_INVALID;
  if (n_missions < 1 || n_missions > kMaxMissions || !missions || !d_v || !stats || max_sweeps < 0) {
    set_err(ctx, "n_missions must be in [1, %d]; missions, d_v and stats non-NULL; max_sweeps >= 0", kMaxMissions);
    return MDP_E_INVALID;
  }
  Plan pl;
  MultiVI M;
  memset(&M, 0, sizeof(M));
  M.m = n_missions;
  for (int i = 0; i < n_missions; ++i) {
    mdp_status rc = vi_setup(ctx, p, model, missions[i], pl, M.d[i].P);
    if (rc != MDP_OK) return rc;
    for (int j = 0; j < i; ++j)
      if (missions[j] == missions[i] || d_v[j] == d_v[i]) {
        set_err(ctx, "missions and value buffers must be distinct");
        return MDP_E_INVALID;
      }
    if (!is_device_ptr(d_v[i])) {
      set_err(ctx, "d_v[%d] must be a device pointer", i);
      return MDP_E_INVALID;
    }
  }
  const size_t need = (size_t)n_missions * pl.vi_bytes;
  if (!is_device_ptr(scratch) || scratch_bytes < need) {
    set_err(ctx, "scratch needs %zu device bytes", need);
    return MDP_E_SCRATCH;
  }
  // [sweep states][stats][per-block residuals][second value buffer per mission]
  char *sc = (char *)scratch;
  size_t off = 0;
  VIState *st = (VIState *)(sc + off);
  off = align_up(off + sizeof(VIState) * n_missions);
  mdp_vi_stats *dstats = (mdp_vi_stats *)(sc + off);
  off = align_up(off + sizeof(mdp_vi_stats) * n_missions);
  double *wg_res = (double *)(sc + off);
  off = align_up(off + sizeof(double) * kViGridMaxHost * n_missions);
  for (int i = 0; i < n_missions; ++i) {
    BatchVIDesc &d = M.d[i];
    d.st = d.P.st = st + i;
    d.P.tol = tol;
    d.v = d_v[i];
    d.v_alt = (double *)(sc + off);
    off = align_up(off + (size_t)d.P.ns * 8);
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = launch_vi_init(st, n_missions, s)) != hipSuccess) return hip_fail(ctx, e, "vi init");
  int n = max_sweeps;
  if (tol > 0.0) n = std::min(n, p->nt + 1);  // layered: converged after nt + 1 sweeps
  for (int k = 0; k < n; ++k) {
    Timed tm(ctx, MDP_KERNEL_VI_SWEEP, s);
    if ((e = launch_vi_sweep_missions(M, vi_active_layers(p->nt, k), wg_res, tol, s)) != hipSuccess)
      return hip_fail(ctx, e, "vi sweep");
  }
  if ((e = launch_vi_finish_missions(M, dstats, s)) != hipSuccess) return hip_fail(ctx, e, "vi finish");
  if ((e = hipMemcpyAsync(stats, dstats, sizeof(mdp_vi_stats) * n_missions, hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return hip_fail(ctx, e, "vi stats copy");
  return MDP_OK;
}

mdp_status mdp_policy(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                      const double *d_v, int32_t *d_pi, void *stream)
{
  Plan pl;
  VIParams V;
  mdp_status rc = vi_setup(ctx, p, model, mission, pl, V);
  if (rc != MDP_OK) return rc;
  if (!is_device_ptr(d_v) || !is_device_ptr(d_pi)) {
    set_err(ctx, "d_v and d_pi must be device pointers");
    return MDP_E_INVALID;
  }
  Timed tm(ctx, MDP_KERNEL_POLICY, (hipStream_t)stream);
  hipError_t e = launch_policy(V, d_v, d_pi, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "policy");
  return MDP_OK;
}

mdp_status mdp_rollout_query(const mdp_problem *p, size_t *scratch_bytes)
{
  if (!scratch_bytes) return MDP_E_INVALID;
  if (check_problem(p)) return MDP_E_INVALID;
  *scratch_bytes = align_up(sizeof(mdp_rollout_stats)) + align_up(sizeof(mdp_rollout_path) * (size_t)p->n_real);
  return MDP_OK;
}

mdp_status mdp_rollout(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const int32_t *d_pi,
                       int32_t *d_traj, mdp_rollout_path *d_paths, void *scratch, size_t scratch_bytes,
                       mdp_rollout_stats *stats, void *stream)
{
  if (!ctx) return MDP_E_INVALID;
  if (const char *e = check_problem(p)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  mdp_problem q = *p;
  q.mission_mask &= ~(1u << MDP_MISSION_NET_ENERGY);  // gbar is optional here
  if (q.mission_mask == 0) q.mission_mask = 1u;
  if (const char *e = check_env(&q, env)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (p->start_i < 0 || p->start_i >= p->nx || p->start_j < 0 || p->start_j >= p->ny) {
    set_err(ctx, "start outside the grid");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(d_pi) || (d_traj && !is_device_ptr(d_traj)) || (d_paths && !is_device_ptr(d_paths)) ||
      !stats) {
    set_err(ctx, "d_pi, d_traj and d_paths must be device pointers (d_traj, d_paths may be NULL), stats non-NULL");
    return MDP_E_INVALID;
  }
  size_t need = 0;
  (void)mdp_rollout_query(p, &need);
  if (!is_device_ptr(scratch) || scratch_bytes < need) {
    set_err(ctx, "scratch needs %zu device bytes", need);
    return MDP_E_SCRATCH;
  }
  RollParams R;
  memset(&R, 0, sizeof(R));
  R.ubar = env->ubar;
  R.vbar = env->vbar;
  R.phiu = env->phiu;
  R.phiv = env->phiv;
  R.mu = env->mu;
  R.gbar = env->gbar;
  R.mask = env->mask;
  R.pi = d_pi;
  R.traj = d_traj;
  mdp_rollout_stats *dstats = (mdp_rollout_stats *)scratch;
  R.paths = d_paths ? d_paths : (mdp_rollout_path *)((char *)scratch + align_up(sizeof(mdp_rollout_stats)));
  R.nx = p->nx;
  R.ny = p->ny;
  R.nt = p->nt;
  R.nc = p->nx * p->ny;
  R.nr = p->n_real;
  R.K = p->n_modes;
  R.na = p->n_head * p->n_speed;
  R.si = p->start_i;
  R.sj = p->start_j;
  R.ti = p->target_i;
  R.tj = p->target_j;
  R.mean_tstride = p->mean_time_varying ? R.nc : 0;
  R.mode_tstride = p->mode_time_varying ? (int64_t)p->n_modes * R.nc : 0;
  R.lam_x = (float)(p->dt / p->dx);
  R.lam_y = (float)(p->dt / p->dy);
  R.swept = (p->flags & MDP_FLAG_SWEPT_PATH) ? 1 : 0;
  R.dt = p->dt;
  R.r_term = p->r_term;
  R.r_out = p->r_outbound;
  R.c_f = p->c_f;
  R.c_r = p->c_r;
  action_tables(p, R.tab.hx, R.tab.hy);
  for (int jf = 0; jf < p->n_speed; ++jf)
    for (int h = 0; h < p->n_head; ++h) R.speed[jf * p->n_head + h] = p->f_max * (double)(jf + 1) / (double)p->n_speed;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_rollout(R, dstats, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "rollout");
  if ((e = hipMemcpyAsync(stats, dstats, sizeof(mdp_rollout_stats), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(ctx, e, "rollout stats copy");
  return MDP_OK;
}

}  // extern "C"

// ====================================================================== batches
namespace {

constexpr int kBatchViGrid = 8192;

struct BatchLayout {
  size_t st, bstats, ctr, vst, vstats, wg_res, pool, total;
  std::vector<size_t> row_nnz, row_off, item_total, item_base, item_off, v_alt;
};

const char *batch_layout(int n, const mdp_problem *probs, int64_t pool_entries, std::vector<Plan> &plans,
                         BatchLayout &L, int64_t &pool_cap, const mdp_ctx *ctx = nullptr)
{
  if (n < 1 || n > kMaxBatch) return "batch size must be in [1, 1024]";
  plans.resize(n);
  int64_t rows_all = 0;
  for (int i = 0; i < n; ++i) {
    if (const char *e = ctx_plan(ctx, &probs[i], plans[i])) return e;
    rows_all += plans[i].rows;
  }
  pool_cap = pool_entries > 0 ? pool_entries : 4 * rows_all + 1024;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.st = take(sizeof(BuildState) * n);
  L.bstats = take(sizeof(mdp_build_stats) * n);
  L.ctr = take(4 * kMaxBuildLaunches + 8);  // group work counters, staging pool top
  L.vst = take(sizeof(VIState) * n);
  L.vstats = take(sizeof(mdp_vi_stats) * n);
  L.wg_res = take(sizeof(double) * (size_t)kBatchViGrid * n);
  L.row_nnz.resize(n);
  L.row_off.resize(n);
  L.item_total.resize(n);
  L.item_base.resize(n);
  L.item_off.resize(n);
  L.v_alt.resize(n);
  for (int i = 0; i < n; ++i) {
    const Plan &pl = plans[i];
    const size_t items = (size_t)probs[i].nt * max_tiles_per_layer(&probs[i]);  // any launch shape
    L.row_nnz[i] = take(4 * (size_t)pl.rows);
    L.row_off[i] = take(4 * (size_t)pl.rows);
    L.item_total[i] = take(4 * items);
    L.item_base[i] = take(8 * items);
    L.item_off[i] = take(8 * items);
    L.v_alt[i] = take(8 * (size_t)probs[i].nt * pl.nc);
  }
  L.pool = take(8 * (size_t)pool_cap);
  L.total = off;
  return nullptr;
}

// Per-problem scratch of a batched build, device addresses.
struct BuildScratch {
  BuildState *st;
  uint32_t *row_nnz, *row_off, *item_total;
  int64_t *item_base, *item_off;
};

// Build descriptor of one problem of a batch, its action tables (htab:
// 2 * kMaxA floats for d_tab) and its (cost, item) work list entries.
const char *batch_build_desc(int inst, const mdp_problem *p, const mdp_env *env, const mdp_model &M, const Plan &pl,
                             const BuildScratch &B, float *d_tab, float *htab, BatchBuildDesc &D,
                             std::vector<std::pair<double, BatchItem>> &items)
{
  if (const char *m = check_env(p, env)) return m;
  if (p->flags & MDP_FLAG_SWEPT_PATH) return "batches and servers do not take the swept-path test";
  memset(&D, 0, sizeof(D));
  ActionTables T;
  fill_params(p, env, &M, pl, D.P, T);
  double mx = 0.0, my = 0.0;
  for (int a = 0; a < pl.na; ++a) {
    mx = std::max(mx, fabs((double)T.hx[a]));
    my = std::max(my, fabs((double)T.hy[a]));
  }
  if (safe_speed(p->sub_hx, mx, 1.0, p->nx) < 0.0f || safe_speed(p->sub_hy, my, 1.0, p->ny) < 0.0f)
    return "the sub-grid cannot hold the agent's own displacement";
  memcpy(htab, T.hx, sizeof(T.hx));
  memcpy(htab + kMaxA, T.hy, sizeof(T.hy));
  D.P.tab = d_tab;
  D.st = B.st;
  D.row_nnz = B.row_nnz;
  D.row_off = B.row_off;
  D.item_total = B.item_total;
  D.item_base = B.item_base;
  D.item_off = B.item_off;
  D.M = ModelOut{M.row_ptr, M.col, M.cnt, M.nnz_capacity};
  D.n_items = (int64_t)p->nt * pl.tiles_per_layer;
  D.near_asked = (p->flags & MDP_FLAG_NEAR_EDGE) ? 1 : 0;
  for (int t = 0; t < p->nt; ++t)
    for (int tile = 0; tile < pl.tiles_per_layer; ++tile) {
      const int ncell = std::min(pl.cells_per_tile, pl.nc - tile * pl.cells_per_tile);
      const double cost = (double)ncell * p->n_real * (pl.na + 0.25 * p->n_modes);
      items.push_back({cost, BatchItem{inst, t, tile, 0}});
    }
  return nullptr;
}

// Solve descriptor of one problem of a batch.
void batch_vi_desc(const mdp_problem *p, const mdp_model &M, const Plan &pl, int mission, double *v, double *v_alt,
                   int32_t *pi, VIState *st, BatchVIDesc &V)
{
  memset(&V, 0, sizeof(V));
  fill_vi_params(p, &M, pl, mission, kBatchViGrid, V.P);
  V.st = st;
  V.P.st = st;
  V.v = v;
  V.v_alt = v_alt;
  V.pi = pi;
}

// LDS bytes of the widest v window among the problems of a batched sweep.
size_t batch_win_bytes(const BatchVIDesc *vd, int n)
{
  size_t w = 0;
  for (int i = 0; i < n; ++i) w = std::max(w, (size_t)vd[i].P.win_rows * vd[i].P.nx * 8);
  return w;
}

// Persistent-build grid: resident workgroups of the device, at most one per item.
hipError_t batch_build_grid(int kmax, bool near, size_t lds, int n_items, int *grid)
{
  int per_cu = 0;
  hipError_t e = batch_build_occupancy(kmax, near, lds, &per_cu);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidValue;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  *grid = std::max(1, std::min(per_cu * std::max(cus, 1), n_items));
  return hipSuccess;
}

// One persistent launch of a batched build: problems sharing a kernel variant.
struct BuildGroup {
  int kmax = 4;
  bool near = false;
  int occ = 0;  // workgroups per CU that the LDS allows
  size_t lds = 0;
  int first = 0, count = 0, grid = 1;
};

// Order the work list by group (mode bound, near-edge counting) and, inside a
// group, by descending cost; fill each group's item range and grid.
hipError_t plan_build_groups(std::vector<std::pair<double, BatchItem>> &items, const std::vector<int> &kmax_of,
                             const std::vector<char> &near_of, const std::vector<size_t> &lds_of,
                             std::vector<BatchItem> &flat, std::vector<BuildGroup> &groups, int share_pct = 100,
                             std::vector<double> *flat_cost = nullptr)
{
  const int n = (int)kmax_of.size();
  std::vector<int> gid(n);
  groups.clear();
  for (int i = 0; i < n; ++i) {
    // problems whose histograms allow the same number of resident workgroups
    // share a launch, so no problem runs at a larger problem's occupancy
    const int occ = (int)std::min<size_t>(8, kLdsLimit / std::max<size_t>(lds_of[i], 1));
    int g = 0;
    while (g < (int)groups.size() &&
           !(groups[g].kmax == kmax_of[i] && groups[g].near == (near_of[i] != 0) && groups[g].occ == occ))
      ++g;
    if (g == (int)groups.size()) {
      if ((int)groups.size() == kMaxBuildGroups) return hipErrorInvalidValue;
      BuildGroup G;
      G.kmax = kmax_of[i];
      G.near = near_of[i] != 0;
      G.occ = occ;
      groups.push_back(G);
    }
    groups[g].lds = std::max(groups[g].lds, lds_of[i]);
    gid[i] = g;
  }
  std::stable_sort(items.begin(), items.end(),
                   [&](const std::pair<double, BatchItem> &x, const std::pair<double, BatchItem> &y) {
                     const int gx = gid[x.second.inst], gy = gid[y.second.inst];
                     return gx != gy ? gx < gy : x.first > y.first;
                   });
  flat.resize(items.size());
  for (size_t k = 0; k < items.size(); ++k) flat[k] = items[k].second;
  if (flat_cost) {
    flat_cost->resize(items.size());
    for (size_t k = 0; k < items.size(); ++k) (*flat_cost)[k] = items[k].first;
  }
  for (size_t k = 0; k < flat.size(); ++k) {
    BuildGroup &G = groups[gid[flat[k].inst]];
    if (G.count == 0) G.first = (int)k;
    ++G.count;
  }
  for (BuildGroup &G : groups) {
    hipError_t e = batch_build_grid(G.kmax, G.near, G.lds, std::max(G.count, 1), &G.grid);
    if (e != hipSuccess) return e;
    if (share_pct > 0 && share_pct < 100) G.grid = std::max(1, (int)((int64_t)G.grid * share_pct / 100));
  }
  return hipSuccess;
}

// Enqueue the persistent launches of a batched build (after its init kernel):
// one per group, or, when item_cost is given, consecutive chunks of at most
// max_cost each (so that work on other streams can run between them).
// One persistent launch over items [first, first + count) of a group.
struct BuildLaunch {
  int first = 0, count = 0, kmax = 4, grid = 1, counter = 0;
  bool near = false;
  size_t lds = 0;
};

// The launches of a work list: one per group, or, with item costs and
// max_cost > 0, runs of consecutive items of at most max_cost each (while
// launch counters last).
std::vector<BuildLaunch> plan_build_launches(const std::vector<BuildGroup> &groups,
                                             const std::vector<double> *item_cost = nullptr, double max_cost = 0.0)
{
  std::vector<BuildLaunch> out;
  int launch = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    const BuildGroup &G = groups[g];
    int k = G.first;
    const int end = G.first + G.count;
    while (k < end) {
      int k1 = end;
      if (item_cost && max_cost > 0.0 && kMaxBuildLaunches - launch > (int)(groups.size() - g)) {
        double c = 0.0;
        k1 = k;
        while (k1 < end && (k1 == k || c + (*item_cost)[k1] <= max_cost)) c += (*item_cost)[k1++];
      }
      if (launch == kMaxBuildLaunches - 1) k1 = end;  // the last counter takes the rest
      BuildLaunch b;
      b.first = k;
      b.count = k1 - k;
      b.kmax = G.kmax;
      b.near = G.near;
      b.lds = G.lds;
      b.grid = std::min(G.grid, k1 - k);
      b.counter = launch++;
      out.push_back(b);
      k = k1;
    }
  }
  return out;
}

hipError_t enqueue_build_launch(mdp_ctx *ctx, const BatchBuildDesc *D, const BatchItem *d_items, const BuildLaunch &b,
                                unsigned int *counters, uint64_t *pool, unsigned long long *pool_top,
                                int64_t pool_cap, hipStream_t s)
{
  Timed tm(ctx, MDP_KERNEL_BUILD, s);
  return launch_batch_build(D, d_items + b.first, b.count, counters + b.counter, pool, pool_top, pool_cap, b.kmax,
                            b.near, b.lds, b.grid, s);
}

hipError_t enqueue_build_groups(mdp_ctx *ctx, const BatchBuildDesc *D, const BatchItem *d_items,
                                const std::vector<BuildGroup> &groups, unsigned int *counters, uint64_t *pool,
                                unsigned long long *pool_top, int64_t pool_cap, hipStream_t s)
{
  for (const BuildLaunch &b : plan_build_launches(groups)) {
    hipError_t e = enqueue_build_launch(ctx, D, d_items, b, counters, pool, pool_top, pool_cap, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per-sweep tables of the blocks each problem recomputes: table j (n + 1
// entries) for problems that have sweeps[i] + j sweeps behind them.
void active_block_tables(const BatchVIDesc *vd, const int *sweeps, int n, int n_tables, std::vector<int64_t> &out)
{
  out.assign((size_t)n_tables * (n + 1), 0);
  for (int j = 0; j < n_tables; ++j) {
    int64_t *tab = &out[(size_t)j * (n + 1)];
    for (int i = 0; i < n; ++i)
      tab[i + 1] = tab[i] + (int64_t)vi_active_layers(vd[i].P.nt, sweeps[i] + j) * vd[i].P.blocks_per_layer;
  }
}

}  // namespace

struct mdp_batch {
  mdp_ctx *ctx = nullptr;
  int n = 0;
  std::vector<BuildGroup> groups;
  int n_items = 0;
  int max_nt = 0;
  int64_t pool_cap = 0;
  size_t win_bytes = 0;  // widest v window of the solve
  char *scratch = nullptr;
  BatchLayout L;
  BatchBuildDesc *d_bdesc = nullptr;
  BatchVIDesc *d_vdesc = nullptr;
  BatchItem *d_items = nullptr;
  float *d_tabs = nullptr;
  int64_t *d_block_start = nullptr;  // every block of every problem (policy)
  int64_t *d_bs_sweeps = nullptr;    // [max_nt + 2][n + 1]: blocks recomputed by sweep k
  hipGraphExec_t gexec = nullptr;
};

extern "C" {

mdp_status mdp_batch_query(int32_t n, const mdp_problem *probs, int64_t pool_entries, size_t *scratch_bytes)
{
  if (!probs || !scratch_bytes) return MDP_E_INVALID;
  std::vector<Plan> plans;
  BatchLayout L;
  int64_t cap;
  if (batch_layout(n, probs, pool_entries, plans, L, cap)) return MDP_E_INVALID;
  *scratch_bytes = L.total;
  return MDP_OK;
}

static void batch_free(mdp_batch *b)
{
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->d_bdesc) (void)hipFree(b->d_bdesc);
  if (b->d_vdesc) (void)hipFree(b->d_vdesc);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_tabs) (void)hipFree(b->d_tabs);
  if (b->d_block_start) (void)hipFree(b->d_block_start);
  if (b->d_bs_sweeps) (void)hipFree(b->d_bs_sweeps);
  delete b;
}

mdp_status mdp_batch_create(mdp_ctx *ctx, int32_t n, const mdp_problem *probs, const mdp_env *envs,
                            const mdp_model *models, const int32_t *missions, double *const *d_v,
                            int32_t *const *d_pi, int64_t pool_entries, void *scratch, size_t scratch_bytes,
                            mdp_batch **out)
{
  if (!ctx || !probs || !envs || !models || !missions || !d_v || !d_pi || !out) return MDP_E_INVALID;
  *out = nullptr;
  std::vector<Plan> plans;
  BatchLayout L;
  int64_t pool_cap = 0;
  if (const char *e = batch_layout(n, probs, pool_entries, plans, L, pool_cap, ctx)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(scratch) || scratch_bytes < L.total) {
    set_err(ctx, "batch scratch needs %zu device bytes", L.total);
    return MDP_E_SCRATCH;
  }
  std::vector<BatchBuildDesc> bd(n);
  std::vector<BatchVIDesc> vd(n);
  std::vector<float> tabs((size_t)n * 2 * kMaxA, 0.0f);
  std::vector<int64_t> block_start(n + 1, 0);
  std::vector<std::pair<double, BatchItem>> items;
  std::vector<int> kmax_of(n);
  std::vector<char> near_of(n);
  std::vector<size_t> lds_of(n);
  mdp_batch *b = new mdp_batch();
  b->ctx = ctx;
  b->n = n;
  b->L = L;
  b->pool_cap = pool_cap;
  b->scratch = (char *)scratch;
  char *sc = (char *)scratch;
  hipError_t e = hipMalloc((void **)&b->d_tabs, sizeof(float) * tabs.size());
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(ctx, e, "batch tables");
  }
  for (int i = 0; i < n; ++i) {
    const mdp_problem *p = &probs[i];
    const Plan &pl = plans[i];
    const mdp_model &M = models[i];
    if (!is_device_ptr(M.row_ptr) || !is_device_ptr(M.reward) || !is_device_ptr(M.col) || !is_device_ptr(M.cnt) ||
        !is_device_ptr(d_v[i]) || !is_device_ptr(d_pi[i])) {
      set_err(ctx, "problem %d: model, value and policy buffers must be device pointers", i);
      batch_free(b);
      return MDP_E_INVALID;
    }
    const int mission = missions[i];
    if (mission < 0 || mission > 2 || !(p->mission_mask >> mission & 1u)) {
      set_err(ctx, "problem %d: mission %d is not built", i, mission);
      batch_free(b);
      return MDP_E_INVALID;
    }
    const BuildScratch B{(BuildState *)(sc + L.st) + i,         (uint32_t *)(sc + L.row_nnz[i]),
                         (uint32_t *)(sc + L.row_off[i]),       (uint32_t *)(sc + L.item_total[i]),
                         (int64_t *)(sc + L.item_base[i]),      (int64_t *)(sc + L.item_off[i])};
    if (const char *m = batch_build_desc(i, p, &envs[i], M, pl, B, b->d_tabs + (size_t)i * 2 * kMaxA,
                                         &tabs[(size_t)i * 2 * kMaxA], bd[i], items)) {
      set_err(ctx, "problem %d: %s", i, m);
      batch_free(b);
      return MDP_E_INVALID;
    }
    kmax_of[i] = pl.kmax;
    near_of[i] = (char)bd[i].near_asked;
    lds_of[i] = pl.lds;
    b->max_nt = std::max(b->max_nt, p->nt);
    batch_vi_desc(p, M, pl, mission, d_v[i], (double *)(sc + L.v_alt[i]), d_pi[i], (VIState *)(sc + L.vst) + i,
                  vd[i]);
    block_start[i + 1] = block_start[i] + vd[i].P.n_blocks;
  }
  std::vector<BatchItem> flat;
  if ((e = plan_build_groups(items, kmax_of, near_of, lds_of, flat, b->groups)) != hipSuccess) {
    batch_free(b);
    return hip_fail(ctx, e, "batch occupancy");
  }
  b->n_items = (int)flat.size();
  b->win_bytes = batch_win_bytes(vd.data(), n);
  std::vector<int64_t> bs_sweeps;
  const std::vector<int> zero(n, 0);
  active_block_tables(vd.data(), zero.data(), n, b->max_nt + 2, bs_sweeps);
  if ((e = hipMalloc((void **)&b->d_bdesc, sizeof(BatchBuildDesc) * n)) != hipSuccess ||
      (e = hipMalloc((void **)&b->d_vdesc, sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = hipMalloc((void **)&b->d_items, sizeof(BatchItem) * flat.size())) != hipSuccess ||
      (e = hipMalloc((void **)&b->d_block_start, sizeof(int64_t) * (n + 1))) != hipSuccess ||
      (e = hipMalloc((void **)&b->d_bs_sweeps, sizeof(int64_t) * bs_sweeps.size())) != hipSuccess ||
      (e = hipMemcpy(b->d_bs_sweeps, bs_sweeps.data(), sizeof(int64_t) * bs_sweeps.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(b->d_bdesc, bd.data(), sizeof(BatchBuildDesc) * n, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_vdesc, vd.data(), sizeof(BatchVIDesc) * n, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_items, flat.data(), sizeof(BatchItem) * flat.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_block_start, block_start.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(b->d_tabs, tabs.data(), sizeof(float) * tabs.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    batch_free(b);
    return hip_fail(ctx, e, "batch descriptors");
  }
  *out = b;
  return MDP_OK;
}

mdp_status mdp_batch_build(mdp_batch *b, void *stream)
{
  if (!b) return MDP_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  char *sc = b->scratch;
  unsigned int *counter = (unsigned int *)(sc + b->L.ctr);  // one per group
  unsigned long long *pool_top = (unsigned long long *)(sc + b->L.ctr + 4 * kMaxBuildLaunches);
  uint64_t *pool = (uint64_t *)(sc + b->L.pool);
  hipError_t e;
  if ((e = launch_batch_build_init(b->d_bdesc, b->n, counter, pool_top, s)) != hipSuccess)
    return hip_fail(b->ctx, e, "batch init");
  if ((e = enqueue_build_groups(b->ctx, b->d_bdesc, b->d_items, b->groups, counter, pool, pool_top, b->pool_cap,
                                 s)) != hipSuccess)
    return hip_fail(b->ctx, e, "batch build");
  if ((e = launch_batch_scan(b->d_bdesc, b->n, s)) != hipSuccess) return hip_fail(b->ctx, e, "batch scan");
  {
    Timed tm(b->ctx, MDP_KERNEL_COPY, s);
    if ((e = launch_batch_copy(b->d_bdesc, b->d_items, b->n_items, pool, s)) != hipSuccess)
      return hip_fail(b->ctx, e, "batch copy");
  }
  if ((e = launch_batch_finalize(b->d_bdesc, b->n, (mdp_build_stats *)(sc + b->L.bstats), s)) != hipSuccess)
    return hip_fail(b->ctx, e, "batch finalize");
  return MDP_OK;
}

mdp_status mdp_batch_solve(mdp_batch *b, double tol, int32_t max_sweeps, void *stream)
{
  if (!b || max_sweeps < 0) return MDP_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  char *sc = b->scratch;
  double *wg_res = (double *)(sc + b->L.wg_res);
  hipError_t e;
  // cold start of every problem: v = 0 and a fresh sweep state (a kernel, so
  // that a captured graph resets them on every replay)
  if ((e = launch_vi_reset_batched(b->d_vdesc, b->n, s)) != hipSuccess) return hip_fail(b->ctx, e, "vi reset");
  int sweeps = max_sweeps;
  if (tol > 0.0) sweeps = std::min(sweeps, b->max_nt + 1);
  for (int k = 0; k < sweeps; ++k) {
    Timed tm(b->ctx, MDP_KERNEL_VI_SWEEP, s);
    if ((e = launch_vi_sweep_batched(b->d_vdesc, b->n, b->d_bs_sweeps + (size_t)std::min(k, b->max_nt + 1) * (b->n + 1),
                                       wg_res, kBatchViGrid, b->win_bytes, s)) !=
        hipSuccess)
      return hip_fail(b->ctx, e, "batch sweep");
    if ((e = launch_vi_close_batched(b->d_vdesc, b->n, kBatchViGrid, wg_res, tol, s)) != hipSuccess)
      return hip_fail(b->ctx, e, "batch close");
  }
  if ((e = launch_vi_finish_batched(b->d_vdesc, b->n, (mdp_vi_stats *)(sc + b->L.vstats), s)) != hipSuccess)
    return hip_fail(b->ctx, e, "batch finish");
  Timed tm(b->ctx, MDP_KERNEL_POLICY, s);
  if ((e = launch_policy_batched(b->d_vdesc, b->n, b->d_block_start, kBatchViGrid, b->win_bytes, s)) != hipSuccess)
    return hip_fail(b->ctx, e, "batch policy");
  return MDP_OK;
}

mdp_status mdp_batch_stats(mdp_batch *b, mdp_build_stats *build_stats, mdp_vi_stats *vi_stats)
{
  if (!b) return MDP_E_INVALID;
  hipError_t e;
  if (build_stats &&
      (e = hipMemcpy(build_stats, b->scratch + b->L.bstats, sizeof(mdp_build_stats) * b->n, hipMemcpyDeviceToHost)) !=
          hipSuccess)
    return hip_fail(b->ctx, e, "batch stats");
  if (vi_stats &&
      (e = hipMemcpy(vi_stats, b->scratch + b->L.vstats, sizeof(mdp_vi_stats) * b->n, hipMemcpyDeviceToHost)) !=
          hipSuccess)
    return hip_fail(b->ctx, e, "batch stats");
  return MDP_OK;
}

mdp_status mdp_batch_capture(mdp_batch *b, double tol, int32_t max_sweeps, void *stream)
{
  if (!b || !stream) return MDP_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  const bool prof = b->ctx->profiling;
  b->ctx->profiling = false;  // no event records inside the graph
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    b->ctx->profiling = prof;
    return hip_fail(b->ctx, e, "begin capture");
  }
  mdp_status rc = mdp_batch_build(b, stream);
  if (rc == MDP_OK) rc = mdp_batch_solve(b, tol, max_sweeps, stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  b->ctx->profiling = prof;
  if (rc != MDP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(b->ctx, e, "end capture");
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec = nullptr;
    return hip_fail(b->ctx, e, "graph instantiate");
  }
  return MDP_OK;
}

mdp_status mdp_batch_replay(mdp_batch *b, void *stream)
{
  if (!b || !b->gexec) return MDP_E_INVALID;
  hipError_t e = hipGraphLaunch(b->gexec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(b->ctx, e, "graph launch");
  return MDP_OK;
}

mdp_status mdp_batch_destroy(mdp_batch *b)
{
  if (!b) return MDP_E_INVALID;
  batch_free(b);
  return MDP_OK;
}

}  // extern "C"

// ====================================================================== serving
namespace {

// First-fit allocator over one caller-owned device range (host bookkeeping only).
class RangeAlloc {
 public:
  void reset(size_t cap)
  {
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t &off)
  {
    bytes = align_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes)
  {
    bytes = align_up(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // Keep the first new_bytes of a block of old_bytes; the tail becomes free.
  void shrink(size_t off, size_t old_bytes, size_t new_bytes)
  {
    const size_t a = align_up(std::max<size_t>(old_bytes, 1)), b = align_up(std::max<size_t>(new_bytes, 1));
    if (b < a) release(off + b, a - b);
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length, disjoint and non-adjacent
  size_t used_ = 0;
};

struct Block {
  size_t off = 0, len = 0;
  bool live = false;
};

// Pool bytes a request holds from admission until its build is checked:
// model with the worst-case nonzeros, values, policy, sweep state, and its
// share of the build scratch and staging pool.
struct ReqSizes {
  int64_t rows, ns, cap;
  size_t keep, col, cnt, build;
};

ReqSizes req_sizes(const mdp_problem *p, const Plan &pl)
{
  ReqSizes z;
  z.rows = pl.rows;
  z.ns = (int64_t)p->nt * pl.nc;
  z.cap = pl.rows * (int64_t)pl.max_row;
  z.keep = align_up(8 * (size_t)(z.rows + 1)) + align_up(4 * (size_t)z.rows) + 2 * align_up(8 * (size_t)z.ns) +
           align_up(4 * (size_t)z.ns) + align_up(sizeof(VIState));
  z.col = align_up(4 * (size_t)z.cap);
  z.cnt = align_up(2 * (size_t)z.cap);
  const size_t items = (size_t)p->nt * max_tiles_per_layer(p);
  z.build = align_up(sizeof(BuildState)) + align_up(sizeof(mdp_build_stats)) + 2 * align_up(4 * (size_t)z.rows) +
            align_up(4 * items) + 2 * align_up(8 * items) + align_up(sizeof(BatchItem) * items) +
            align_up(8 * (size_t)z.cap);
  return z;
}

struct ServeReq {
  int64_t tag = 0;
  int64_t seq = 0;  // submission order
  mdp_problem p{};
  mdp_env env{};
  int mission = 0;
  int32_t *h_pi = nullptr;
  double *h_v = nullptr;
  Plan pl{};
  ReqSizes z{};
  Block keep, col, cnt;
  int64_t model_cap = 0;  // col / cnt entries held: worst case until the build is checked
  bool cold = false;      // built; v and the sweep state are reset at its first step
  int sweeps = 0;         // sweeps enqueued since its first step
  int limit = 0;   // sweeps after which the request retires in any case
  mdp_served res{};
  // addresses inside the pool (valid while admitted)
  int64_t *row_ptr = nullptr;
  float *reward = nullptr;
  double *v = nullptr, *v_alt = nullptr;
  int32_t *pi = nullptr;
  VIState *st = nullptr;
  int32_t *colp = nullptr;
  uint16_t *cntp = nullptr;
};

}  // namespace

// Pinned host staging of one kind of upload or download; it is rewritten only
// after the device work that used it last has completed.
struct Pinned {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes)
  {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc(&p, std::max<size_t>(bytes, 64), hipHostMallocDefault);
    if (e == hipSuccess) n = std::max<size_t>(bytes, 64);
    return e;
  }
  template <typename T>
  T *as() const
  {
    return (T *)p;
  }
  ~Pinned()
  {
    if (p) (void)hipHostFree(p);
  }
};

// A build lane: one build batch at a time on a stream of its own. Small and
// large requests use different lanes, so a small build never waits for a
// large one (each large build is split into short launches that the small
// lane's and the sweeps' kernels interleave with).
constexpr int kServeAhead = 2;  // build launches of a lane in flight at once

struct BuildLane {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;       // end of the batch in flight (recorded with its tail)
  std::vector<ServeReq *> building; // the batch in flight
  Block blk;                        // its scratch and staging block
  BatchBuildDesc *d_bdesc = nullptr;
  float *d_tabs = nullptr;
  BatchItem *d_items = nullptr;     // the batch's work list, inside its build block
  Pinned h_bdesc, h_items, h_tabs, h_bstat;
  // The batch's build launches are enqueued a few at a time (serve_pump), so
  // that sweeps enqueued meanwhile on other streams reach the GPU between
  // them instead of behind the whole build.
  std::vector<BuildLaunch> plan;
  size_t next = 0;
  hipEvent_t ahead[kServeAhead] = {};
  int ahead_head = 0, ahead_n = 0;
  bool tail = false;  // scan, copy, statistics and `event` enqueued
  unsigned int *counter = nullptr;
  uint64_t *pool = nullptr;
  unsigned long long *pool_top = nullptr;
  int64_t pool_cap = 0;
  int n_items = 0;
  mdp_build_stats *bstats = nullptr;
  // Large lane only: once its build batch is done, the batch's whole solve
  // runs on the lane's stream (cold start, every sweep a few launches at a
  // time as for the build, finish, policy, results into pinned memory), so a
  // large request neither waits for the caller's steps nor makes the small
  // requests' steps carry its sweeps.
  std::vector<ServeReq *> solving;  // the batch being solved
  Block sblk;                       // its block-start tables, inside the pool
  int64_t *d_stabs = nullptr;       // [solve_k][n + 1] per sweep, then [n + 1] for the policy
  int solve_k = 0, solve_next = 0;  // sweeps to enqueue, enqueued
  bool solve_tail = false;          // finish, policy, copies and solve_ev enqueued
  size_t solve_win = 0;
  hipEvent_t solve_ev = nullptr;
  BatchVIDesc *d_svdesc = nullptr;  // [max_inflight]
  double *d_swg = nullptr;          // [kBatchViGrid][max_inflight]
  mdp_vi_stats *d_sstat = nullptr;  // [max_inflight]
  Pinned h_svdesc, h_stabs, h_sfstat, h_svstart;
};

constexpr int kServeLanes = 2;  // 0: small builds, 1: large builds
constexpr int kServeSolveLane = 1;  // the lane whose batches are solved on their own stream
constexpr int kServeSolveGroup = 8;  // sweeps per pumped launch group of a lane solve

struct mdp_server {
  mdp_ctx *ctx = nullptr;
  mdp_server_config cfg{};
  char *pool = nullptr;
  size_t pool_bytes = 0;
  RangeAlloc alloc;
  std::deque<ServeReq *> queue;     // submitted, not admitted
  BuildLane lane[kServeLanes];
  std::vector<ServeReq *> running;  // built; swept on the caller's stream
  std::vector<mdp_served> done;     // completion records not yet polled
  // A step enqueues its sweeps and returns; a later step reads their status
  // once step_ev has completed. Converged requests wait in to_retire until
  // their retirement (finish, policy, copies) is enqueued, then in retiring
  // until ret_ev has completed.
  bool step_inflight = false;
  hipEvent_t step_ev = nullptr;
  std::vector<ServeReq *> step_run;  // the requests the step in flight sweeps
  std::vector<ServeReq *> to_retire, retiring;
  hipEvent_t ret_ev = nullptr;
  int64_t step_no = 0;
  int64_t n_submitted = 0;
  double chunk_cost = 0.0;  // work of one build launch (cfg.chunk_cost or the default)
  double large_cost = 0.0;  // build cost above which a request takes the large lane
  // device tables, sized for cfg.max_inflight problems
  BatchVIDesc *d_vrun = nullptr, *d_vret = nullptr;
  int64_t *d_bs_ret = nullptr;
  int64_t *d_bs_sweeps = nullptr;  // [sweeps_per_step][max_inflight + 1]
  double *d_wg_res = nullptr;
  mdp_vi_stats *d_vstat = nullptr;
  // pinned staging
  Pinned h_vrun, h_tables, h_vstat, h_vret, h_bsret, h_fstat, h_vstart;
  size_t n_building() const
  {
    size_t k = 0;
    for (const BuildLane &L : lane) k += L.building.size();
    return k;
  }
  size_t n_solving() const
  {
    size_t k = 0;
    for (const BuildLane &L : lane) k += L.solving.size();
    return k;
  }
};

namespace {

void serve_free_all(mdp_server *S)
{
  for (BuildLane &L : S->lane) {
    if (L.stream && (!L.building.empty() || !L.solving.empty())) (void)hipStreamSynchronize(L.stream);
    for (ServeReq *r : L.building) delete r;
    for (ServeReq *r : L.solving) delete r;
    for (hipEvent_t ev : L.ahead)
      if (ev) (void)hipEventDestroy(ev);
    void *bufs[] = {L.d_bdesc, L.d_tabs, L.d_svdesc, L.d_swg, L.d_sstat};
    for (void *p : bufs)
      if (p) (void)hipFree(p);
    if (L.event) (void)hipEventDestroy(L.event);
    if (L.solve_ev) (void)hipEventDestroy(L.solve_ev);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  if (S->step_ev) {
    if (S->step_inflight) (void)hipEventSynchronize(S->step_ev);
    (void)hipEventDestroy(S->step_ev);
  }
  if (S->ret_ev) {
    if (!S->retiring.empty()) (void)hipEventSynchronize(S->ret_ev);
    (void)hipEventDestroy(S->ret_ev);
  }
  for (ServeReq *r : S->queue) delete r;
  for (ServeReq *r : S->running) delete r;
  for (ServeReq *r : S->to_retire) delete r;
  for (ServeReq *r : S->retiring) delete r;
  void *bufs[] = {S->d_vrun, S->d_vret, S->d_bs_ret, S->d_bs_sweeps, S->d_wg_res, S->d_vstat};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  delete S;
}

bool take(RangeAlloc &A, Block &b, size_t len)
{
  b.len = len;
  b.live = A.alloc(len, b.off);
  return b.live;
}

void give(RangeAlloc &A, Block &b)
{
  if (b.live) A.release(b.off, b.len);
  b.live = false;
}

// Reserve the model blocks of r and point its buffers into the pool.
bool reserve(mdp_server *S, ServeReq *r)
{
  if (!take(S->alloc, r->keep, r->z.keep)) return false;
  if (!take(S->alloc, r->col, r->z.col)) {
    give(S->alloc, r->keep);
    return false;
  }
  if (!take(S->alloc, r->cnt, r->z.cnt)) {
    give(S->alloc, r->col);
    give(S->alloc, r->keep);
    return false;
  }
  char *k = S->pool + r->keep.off;
  size_t o = 0;
  r->row_ptr = (int64_t *)(k + o);
  o += align_up(8 * (size_t)(r->z.rows + 1));
  r->reward = (float *)(k + o);
  o += align_up(4 * (size_t)r->z.rows);
  r->v = (double *)(k + o);
  o += align_up(8 * (size_t)r->z.ns);
  r->v_alt = (double *)(k + o);
  o += align_up(8 * (size_t)r->z.ns);
  r->pi = (int32_t *)(k + o);
  o += align_up(4 * (size_t)r->z.ns);
  r->st = (VIState *)(k + o);
  r->colp = (int32_t *)(S->pool + r->col.off);
  r->cntp = (uint16_t *)(S->pool + r->cnt.off);
  r->model_cap = r->z.cap;
  return true;
}

void unreserve(mdp_server *S, ServeReq *r)
{
  give(S->alloc, r->cnt);
  give(S->alloc, r->col);
  give(S->alloc, r->keep);
}

mdp_model req_model(const ServeReq *r) { return mdp_model{r->row_ptr, r->colp, r->cntp, r->reward, r->model_cap}; }

constexpr size_t kServeCtrBytes = 4 * kMaxBuildLaunches + 8;  // launch work counters, staging pool top
// Work of one launch of a served build, in the cost unit of the work list
// (landings plus a quarter landing per mode term): about 2 ms on an MI355X,
// so the sweeps of admitted requests interleave with long builds.
constexpr double kServeChunkCost = 6e9;
// A build batch takes the requests behind the first one only while their
// build cost stays within this factor of the first one's.
constexpr double kServeCostRatio = 4.0;
// A step sweeps the requests whose remaining work is within this factor of
// the smallest remaining work.
constexpr double kServeWorkRatio = 4.0;
// Requests above this build cost use the large-build lane (a paper-shaped
// 100 x 100 x 120 request with 5000 realizations and 16 headings is ~1.1e11).
constexpr double kServeLargeCost = 3e10;
// Longest a step waits for a build when it has nothing to sweep.
constexpr int kServeWaitUs = 500;

double build_cost(const ServeReq *r)
{
  return (double)r->z.rows * r->p.n_real * (1.0 + 0.25 * r->p.n_modes / std::max(r->pl.na, 1));
}

size_t build_block_bytes(const std::vector<ServeReq *> &fresh)
{
  size_t b = align_up(kServeCtrBytes) + align_up(sizeof(BuildState) * fresh.size()) +
             align_up(sizeof(mdp_build_stats) * fresh.size());
  for (const ServeReq *r : fresh) b += r->z.build;
  return b;
}

// Keep the lane's build going: enqueue its next launches while fewer than
// kServeAhead are in flight, then, after the last one, the batch's tail (scan,
// copy, statistics into pinned memory, the batch's event).
mdp_status serve_pump(mdp_server *S, BuildLane &L)
{
  hipStream_t s = L.stream;
  hipError_t e;
  while (L.next < L.plan.size()) {
    if (L.ahead_n == kServeAhead) {
      const hipError_t q = hipEventQuery(L.ahead[L.ahead_head]);
      if (q == hipErrorNotReady) return MDP_OK;
      if (q != hipSuccess) return hip_fail(S->ctx, q, "serve build");
      L.ahead_head = (L.ahead_head + 1) % kServeAhead;
      --L.ahead_n;
    }
    if ((e = enqueue_build_launch(S->ctx, L.d_bdesc, L.d_items, L.plan[L.next], L.counter, L.pool, L.pool_top,
                                  L.pool_cap, s)) != hipSuccess ||
        (e = hipEventRecord(L.ahead[(L.ahead_head + L.ahead_n) % kServeAhead], s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve build");
    ++L.ahead_n;
    ++L.next;
  }
  if (L.tail) return MDP_OK;
  const int n = (int)L.building.size();
  if ((e = launch_batch_scan(L.d_bdesc, n, s)) != hipSuccess) return hip_fail(S->ctx, e, "serve scan");
  {
    Timed tm(S->ctx, MDP_KERNEL_COPY, s);
    if ((e = launch_batch_copy(L.d_bdesc, L.d_items, L.n_items, L.pool, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve copy");
  }
  if ((e = launch_batch_finalize(L.d_bdesc, n, L.bstats, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve finalize");
  if ((e = hipMemcpyAsync(L.h_bstat.p, L.bstats, sizeof(mdp_build_stats) * n, hipMemcpyDeviceToHost, s)) !=
          hipSuccess ||
      (e = hipEventRecord(L.event, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve build end");
  L.tail = true;
  return MDP_OK;
}


// Start the batched build of the requests in L.building on the lane's stream:
// descriptors through pinned staging, the work counters, then the persistent
// launches in short chunks, a few at a time (serve_pump).
mdp_status serve_build(mdp_server *S, BuildLane &L, char *blk)
{
  const std::vector<ServeReq *> &fresh = L.building;
  const int n = (int)fresh.size();
  hipStream_t s = L.stream;
  hipError_t e;
  if ((e = L.h_bdesc.ensure(sizeof(BatchBuildDesc) * n)) != hipSuccess ||
      (e = L.h_tabs.ensure(sizeof(float) * 2 * kMaxA * n)) != hipSuccess ||
      (e = L.h_bstat.ensure(sizeof(mdp_build_stats) * n)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve staging");
  BatchBuildDesc *bd = L.h_bdesc.as<BatchBuildDesc>();
  float *tabs = L.h_tabs.as<float>();
  memset(tabs, 0, sizeof(float) * 2 * kMaxA * n);
  std::vector<std::pair<double, BatchItem>> items;
  unsigned int *counter = (unsigned int *)blk;
  unsigned long long *pool_top = (unsigned long long *)(blk + 4 * kMaxBuildLaunches);
  size_t o = align_up(kServeCtrBytes);
  BuildState *st = (BuildState *)(blk + o);
  o += align_up(sizeof(BuildState) * n);
  mdp_build_stats *bstats = (mdp_build_stats *)(blk + o);
  o += align_up(sizeof(mdp_build_stats) * n);
  std::vector<BuildScratch> B(n);
  int64_t pool_cap = 0;
  for (int i = 0; i < n; ++i) {
    const ServeReq *r = fresh[i];
    const size_t items_i = (size_t)r->p.nt * r->pl.tiles_per_layer;
    B[i].st = st + i;
    B[i].row_nnz = (uint32_t *)(blk + o);
    o += align_up(4 * (size_t)r->z.rows);
    B[i].row_off = (uint32_t *)(blk + o);
    o += align_up(4 * (size_t)r->z.rows);
    B[i].item_total = (uint32_t *)(blk + o);
    o += align_up(4 * items_i);
    B[i].item_base = (int64_t *)(blk + o);
    o += align_up(8 * items_i);
    B[i].item_off = (int64_t *)(blk + o);
    o += align_up(8 * items_i);
    pool_cap += r->z.cap;
  }
  size_t n_items_all = 0;
  for (int i = 0; i < n; ++i) n_items_all += (size_t)fresh[i]->p.nt * fresh[i]->pl.tiles_per_layer;
  BatchItem *d_items = (BatchItem *)(blk + o);  // room: every request's z.build holds its items
  o += align_up(sizeof(BatchItem) * n_items_all);
  uint64_t *pool = (uint64_t *)(blk + o);
  std::vector<int> kmax_of(n);
  std::vector<char> near_of(n);
  std::vector<size_t> lds_of(n);
  for (int i = 0; i < n; ++i) {
    ServeReq *r = fresh[i];
    const mdp_model M = req_model(r);
    if (const char *m = batch_build_desc(i, &r->p, &r->env, M, r->pl, B[i], L.d_tabs + (size_t)i * 2 * kMaxA,
                                         &tabs[(size_t)i * 2 * kMaxA], bd[i], items)) {
      set_err(S->ctx, "request %lld: %s", (long long)r->tag, m);
      return MDP_E_INVALID;
    }
    kmax_of[i] = r->pl.kmax;
    near_of[i] = (char)bd[i].near_asked;
    lds_of[i] = r->pl.lds;
  }
  std::vector<BatchItem> flat;
  std::vector<BuildGroup> groups;
  std::vector<double> cost;
  if ((e = plan_build_groups(items, kmax_of, near_of, lds_of, flat, groups, S->cfg.build_share, &cost)) !=
      hipSuccess)
    return hip_fail(S->ctx, e, "serve occupancy");
  if (flat.size() != n_items_all) {
    set_err(S->ctx, "serve work list size");
    return MDP_E_HIP;
  }
  L.d_items = d_items;
  if ((e = L.h_items.ensure(sizeof(BatchItem) * flat.size())) != hipSuccess)
    return hip_fail(S->ctx, e, "serve staging");
  memcpy(L.h_items.p, flat.data(), sizeof(BatchItem) * flat.size());
  if ((e = hipMemcpyAsync(L.d_bdesc, bd, sizeof(BatchBuildDesc) * n, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(L.d_tabs, tabs, sizeof(float) * 2 * kMaxA * n, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(L.d_items, L.h_items.p, sizeof(BatchItem) * flat.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(S->ctx, e, "serve descriptors");
  if ((e = launch_batch_build_init(L.d_bdesc, n, counter, pool_top, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve build init");
  L.plan = plan_build_launches(groups, &cost, S->chunk_cost);
  L.next = 0;
  L.ahead_head = L.ahead_n = 0;
  L.tail = false;
  L.counter = counter;
  L.pool = pool;
  L.pool_top = pool_top;
  L.pool_cap = pool_cap;
  L.n_items = (int)flat.size();
  L.bstats = bstats;
  return serve_pump(S, L);
}

// The build batch has finished: record its statistics, give back the unused
// worst-case reservations and the build block, and let the requests join the
// sweeps (cold start at their first step).
void serve_join(mdp_server *S, BuildLane &L)
{
  const mdp_build_stats *hb = L.h_bstat.as<mdp_build_stats>();
  for (size_t i = 0; i < L.building.size(); ++i) {
    ServeReq *r = L.building[i];
    r->res.nnz = hb[i].nnz;
    r->res.samples = hb[i].samples;
    r->res.build_status = hb[i].status;
    if (hb[i].status == MDP_OK) {
      S->alloc.shrink(r->col.off, r->col.len, 4 * (size_t)hb[i].nnz);
      S->alloc.shrink(r->cnt.off, r->cnt.len, 2 * (size_t)hb[i].nnz);
      r->col.len = align_up(std::max<size_t>(4 * (size_t)hb[i].nnz, 1));
      r->cnt.len = align_up(std::max<size_t>(2 * (size_t)hb[i].nnz, 1));
      r->model_cap = hb[i].nnz;
    }
    r->cold = true;
    S->running.push_back(r);
  }
  L.building.clear();
  give(S->alloc, L.blk);
}

// Lane of a request: large builds (paper-shaped and above) go to lane 1.
int lane_of(const mdp_server *S, const ServeReq *r) { return build_cost(r) > S->large_cost ? 1 : 0; }

// Admit queued requests of lane li's size class, in order, into a new build
// batch while slots and pool space last, and enqueue its build.
mdp_status serve_admit(mdp_server *S, int li)
{
  BuildLane &L = S->lane[li];
  std::vector<ServeReq *> &fresh = L.building;
  Block &bblk = L.blk;
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    if ((int)(S->running.size() + S->to_retire.size() + S->retiring.size() + S->n_building() + S->n_solving()) >=
        S->cfg.max_inflight)
      break;
    ServeReq *r = *it;
    if (lane_of(S, r) != li) {
      ++it;
      continue;
    }
    if (!fresh.empty()) {  // keep a batch's builds within a factor of each other
      const double c0 = build_cost(fresh.front()), c = build_cost(r);
      if (c > kServeCostRatio * c0 || c0 > kServeCostRatio * c) break;
    }
    const size_t prev_len = bblk.live ? bblk.len : 0;
    give(S->alloc, bblk);
    bool ok = reserve(S, r);
    if (ok) {
      fresh.push_back(r);
      ok = take(S->alloc, bblk, build_block_bytes(fresh));
      if (!ok) {
        fresh.pop_back();
        unreserve(S, r);
      }
    }
    if (!ok) {
      if (prev_len && !take(S->alloc, bblk, prev_len)) {  // the range just freed
        set_err(S->ctx, "serve pool bookkeeping");
        return MDP_E_HIP;
      }
      break;
    }
    r->res.admit_step = S->step_no;
    it = S->queue.erase(it);
  }
  if (fresh.empty()) return MDP_OK;
  return serve_build(S, L, S->pool + bblk.off);
}

// Descriptors of reqs into pinned staging vd (returns the widest v window).
size_t vi_descs(const std::vector<ServeReq *> &reqs, BatchVIDesc *vd)
{
  for (size_t i = 0; i < reqs.size(); ++i) {
    ServeReq *r = reqs[i];
    batch_vi_desc(&r->p, req_model(r), r->pl, r->mission, r->v, r->v_alt, r->pi, r->st, vd[i]);
  }
  return batch_win_bytes(vd, (int)reqs.size());
}

// Enqueue the lane solve's sweeps, kServeSolveGroup at a time with at most
// kServeAhead groups in flight, then its tail: finish (values back into v,
// stats), policy, and each request's start value, policy and values into
// pinned host memory, then solve_ev.
mdp_status serve_pump_solve(mdp_server *S, BuildLane &L)
{
  hipStream_t s = L.stream;
  hipError_t e;
  const int n = (int)L.solving.size();
  while (L.solve_next < L.solve_k) {
    if (L.ahead_n == kServeAhead) {
      const hipError_t q = hipEventQuery(L.ahead[L.ahead_head]);
      if (q == hipErrorNotReady) return MDP_OK;
      if (q != hipSuccess) return hip_fail(S->ctx, q, "serve solve");
      L.ahead_head = (L.ahead_head + 1) % kServeAhead;
      --L.ahead_n;
    }
    const int g = std::min(kServeSolveGroup, L.solve_k - L.solve_next);
    for (int j = L.solve_next; j < L.solve_next + g; ++j) {
      Timed tm(S->ctx, MDP_KERNEL_VI_SWEEP, s);
      if ((e = launch_vi_sweep_batched(L.d_svdesc, n, L.d_stabs + (size_t)j * (n + 1), L.d_swg, kBatchViGrid,
                                       L.solve_win, s)) != hipSuccess ||
          (e = launch_vi_close_batched(L.d_svdesc, n, kBatchViGrid, L.d_swg, S->cfg.tol, s)) != hipSuccess)
        return hip_fail(S->ctx, e, "serve solve sweep");
    }
    if ((e = hipEventRecord(L.ahead[(L.ahead_head + L.ahead_n) % kServeAhead], s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve solve");
    ++L.ahead_n;
    L.solve_next += g;
  }
  if (L.solve_tail) return MDP_OK;
  if ((e = launch_vi_finish_batched(L.d_svdesc, n, L.d_sstat, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve solve finish");
  {
    Timed tm(S->ctx, MDP_KERNEL_POLICY, s);
    if ((e = launch_policy_batched(L.d_svdesc, n, L.d_stabs + (size_t)L.solve_k * (n + 1), kBatchViGrid,
                                   L.solve_win, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve solve policy");
  }
  double *vstart = L.h_svstart.as<double>();
  for (int i = 0; i < n; ++i) {
    ServeReq *r = L.solving[i];
    const size_t ns = (size_t)r->z.ns;
    const int64_t s0 = (int64_t)r->p.start_j * r->p.nx + r->p.start_i;
    if ((e = hipMemcpyAsync(&vstart[i], r->v + s0, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (r->h_pi && (e = hipMemcpyAsync(r->h_pi, r->pi, 4 * ns, hipMemcpyDeviceToHost, s)) != hipSuccess) ||
        (r->h_v && (e = hipMemcpyAsync(r->h_v, r->v, 8 * ns, hipMemcpyDeviceToHost, s)) != hipSuccess))
      return hip_fail(S->ctx, e, "serve solve results");
  }
  if ((e = hipMemcpyAsync(L.h_sfstat.p, L.d_sstat, sizeof(mdp_vi_stats) * n, hipMemcpyDeviceToHost, s)) !=
          hipSuccess ||
      (e = hipEventRecord(L.solve_ev, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve solve end");
  L.solve_tail = true;
  return MDP_OK;
}

// The lane's build batch has ended: record its build results and start its
// solve on the lane's stream. Without pool room for the solve's block-start
// tables the batch joins the caller's sweeps instead (serve_join).
mdp_status serve_solve_start(mdp_server *S, BuildLane &L)
{
  const int n = (int)L.building.size();
  int k = 1;
  for (const ServeReq *r : L.building) k = std::max(k, r->limit);
  const size_t tab_bytes = sizeof(int64_t) * (size_t)(n + 1) * (size_t)(k + 1);
  serve_join(S, L);  // build stats, build block and unused model tails back to the pool; batch now in S->running
  if (!take(S->alloc, L.sblk, tab_bytes)) return MDP_OK;
  L.solving.assign(S->running.end() - n, S->running.end());
  S->running.resize(S->running.size() - n);
  hipStream_t s = L.stream;
  hipError_t e;
  if ((e = L.h_svdesc.ensure(sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = L.h_stabs.ensure(tab_bytes)) != hipSuccess ||
      (e = L.h_sfstat.ensure(sizeof(mdp_vi_stats) * n)) != hipSuccess ||
      (e = L.h_svstart.ensure(sizeof(double) * n)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve solve staging");
  BatchVIDesc *vd = L.h_svdesc.as<BatchVIDesc>();
  L.solve_win = vi_descs(L.solving, vd);
  std::vector<int> behind(n, 0);
  std::vector<int64_t> tabs;
  active_block_tables(vd, behind.data(), n, k, tabs);  // cold start: sweep j recomputes layers < nt - j + 1
  tabs.resize((size_t)(n + 1) * (k + 1));
  int64_t *full = &tabs[(size_t)k * (n + 1)];  // every block, for the policy
  full[0] = 0;
  for (int i = 0; i < n; ++i) full[i + 1] = full[i] + vd[i].P.n_blocks;
  memcpy(L.h_stabs.p, tabs.data(), tab_bytes);
  L.d_stabs = (int64_t *)(S->pool + L.sblk.off);
  if ((e = hipMemcpyAsync(L.d_svdesc, vd, sizeof(BatchVIDesc) * n, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(L.d_stabs, L.h_stabs.p, tab_bytes, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = launch_vi_reset_batched(L.d_svdesc, n, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve solve start");
  for (ServeReq *r : L.solving) r->cold = false;
  L.solve_k = k;
  L.solve_next = 0;
  L.solve_tail = false;
  L.ahead_head = L.ahead_n = 0;  // every build launch's event has completed with the build's tail
  return serve_pump_solve(S, L);
}

// The lane's solve has ended: completion records, model memory back to the pool.
void serve_solve_retire(mdp_server *S, BuildLane &L)
{
  const mdp_vi_stats *hf = L.h_sfstat.as<mdp_vi_stats>();
  const double *vstart = L.h_svstart.as<double>();
  for (size_t i = 0; i < L.solving.size(); ++i) {
    ServeReq *r = L.solving[i];
    r->res.sweeps = hf[i].sweeps;
    r->res.residual = hf[i].residual;
    r->res.v_start = vstart[i];
    r->res.status = r->res.build_status != MDP_OK ? r->res.build_status : hf[i].status;
    r->res.done_step = S->step_no;
    S->done.push_back(r->res);
    unreserve(S, r);
    delete r;
  }
  L.solving.clear();
  give(S->alloc, L.sblk);
  L.d_stabs = nullptr;
}

}  // namespace

extern "C" {

mdp_status mdp_server_footprint(const mdp_problem *p, size_t *bytes)
{
  if (!bytes) return MDP_E_INVALID;
  Plan pl;
  if (make_plan(p, pl)) return MDP_E_INVALID;
  const ReqSizes z = req_sizes(p, pl);
  *bytes = z.keep + z.col + z.cnt + z.build + align_up(kServeCtrBytes) + align_up(sizeof(BuildState)) +
           align_up(sizeof(mdp_build_stats));
  return MDP_OK;
}

mdp_status mdp_server_create(mdp_ctx *ctx, const mdp_server_config *cfg, void *pool, size_t pool_bytes,
                             mdp_server **out)
{
  if (!ctx || !cfg || !out) return MDP_E_INVALID;
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxBatch || cfg->sweeps_per_step < 1 ||
      cfg->sweeps_per_step > 256 || cfg->max_sweeps < 1 || cfg->build_share < 0 || cfg->build_share > 100) {
    set_err(ctx, "max_inflight must be in [1, 1024], sweeps_per_step in [1, 256], max_sweeps >= 1, "
                 "build_share in [0, 100]");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(pool) || pool_bytes < kAlign) {
    set_err(ctx, "the model pool must be device memory");
    return MDP_E_INVALID;
  }
  if (!(cfg->chunk_cost >= 0.0) || !(cfg->large_cost >= 0.0)) {
    set_err(ctx, "chunk_cost and large_cost must be >= 0");
    return MDP_E_INVALID;
  }
  mdp_server *S = new mdp_server();
  S->ctx = ctx;
  S->cfg = *cfg;
  S->chunk_cost = cfg->chunk_cost > 0.0 ? cfg->chunk_cost : kServeChunkCost;
  S->large_cost = cfg->large_cost > 0.0 ? cfg->large_cost : kServeLargeCost;
  S->pool = (char *)pool;
  S->pool_bytes = pool_bytes / kAlign * kAlign;
  S->alloc.reset(S->pool_bytes);
  const size_t n = (size_t)cfg->max_inflight;
  const size_t nt = (size_t)cfg->sweeps_per_step;
  hipError_t e;
  for (BuildLane &L : S->lane)
    if ((e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&L.event, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&L.ahead[0], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&L.ahead[1], hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc((void **)&L.d_bdesc, sizeof(BatchBuildDesc) * n)) != hipSuccess ||
        (e = hipMalloc((void **)&L.d_tabs, sizeof(float) * 2 * kMaxA * n)) != hipSuccess) {
      serve_free_all(S);
      return hip_fail(ctx, e, "server build lanes");
    }
  {
    BuildLane &L = S->lane[kServeSolveLane];
    if ((e = hipEventCreateWithFlags(&L.solve_ev, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc((void **)&L.d_svdesc, sizeof(BatchVIDesc) * n)) != hipSuccess ||
        (e = hipMalloc((void **)&L.d_swg, sizeof(double) * kBatchViGrid * n)) != hipSuccess ||
        (e = hipMalloc((void **)&L.d_sstat, sizeof(mdp_vi_stats) * n)) != hipSuccess) {
      serve_free_all(S);
      return hip_fail(ctx, e, "server solve lane");
    }
  }
  if ((e = hipEventCreateWithFlags(&S->step_ev, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&S->ret_ev, hipEventDisableTiming)) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_vrun, sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_vret, sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_bs_ret, sizeof(int64_t) * (n + 1))) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_bs_sweeps, sizeof(int64_t) * (n + 1) * nt)) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_wg_res, sizeof(double) * kBatchViGrid * n)) != hipSuccess ||
      (e = hipMalloc((void **)&S->d_vstat, sizeof(mdp_vi_stats) * n)) != hipSuccess ||
      (e = S->h_vrun.ensure(sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = S->h_tables.ensure(sizeof(int64_t) * (n + 1) * nt)) != hipSuccess ||
      (e = S->h_vstat.ensure(sizeof(mdp_vi_stats) * n)) != hipSuccess ||
      (e = S->h_vret.ensure(sizeof(BatchVIDesc) * n)) != hipSuccess ||
      (e = S->h_bsret.ensure(sizeof(int64_t) * (n + 1))) != hipSuccess ||
      (e = S->h_fstat.ensure(sizeof(mdp_vi_stats) * n)) != hipSuccess ||
      (e = S->h_vstart.ensure(sizeof(double) * n)) != hipSuccess) {
    serve_free_all(S);
    return hip_fail(ctx, e, "server tables");
  }
  *out = S;
  return MDP_OK;
}

mdp_status mdp_server_submit(mdp_server *S, const mdp_problem *p, const mdp_env *env, int32_t mission,
                             int32_t *h_pi, double *h_v, int64_t tag)
{
  if (!S || !p || !env) return MDP_E_INVALID;
  if (mission < 0 || mission > 2) {
    set_err(S->ctx, "mission must be 0, 1 or 2");
    return MDP_E_INVALID;
  }
  if (p->flags & MDP_FLAG_SWEPT_PATH) {
    set_err(S->ctx, "servers do not take the swept-path test");
    return MDP_E_INVALID;
  }
  ServeReq *r = new ServeReq();
  r->tag = tag;
  r->p = *p;
  r->p.mission_mask = 1u << mission;  // one reward block: the requested mission
  r->env = *env;
  r->mission = mission;
  r->h_pi = h_pi;
  r->h_v = h_v;
  if (const char *m = ctx_plan(S->ctx, &r->p, r->pl)) {
    set_err(S->ctx, "request %lld: %s", (long long)tag, m);
    delete r;
    return MDP_E_INVALID;
  }
  if (const char *m = check_env(&r->p, env)) {
    set_err(S->ctx, "request %lld: %s", (long long)tag, m);
    delete r;
    return MDP_E_INVALID;
  }
  r->z = req_sizes(&r->p, r->pl);
  size_t need = 0;
  (void)mdp_server_footprint(&r->p, &need);
  if (need > S->pool_bytes) {
    set_err(S->ctx, "request %lld needs more than the whole pool", (long long)tag);
    delete r;
    return MDP_E_CAPACITY;
  }
  r->limit = S->cfg.max_sweeps;
  if (S->cfg.tol > 0.0) r->limit = std::min(r->limit, r->p.nt + 1);
  r->res.tag = tag;
  r->seq = S->n_submitted++;
  S->queue.push_back(r);
  return MDP_OK;
}

mdp_status mdp_server_step(mdp_server *S, void *stream, int32_t *n_active)
{
  if (!S) return MDP_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  mdp_status rc;
  ++S->step_no;
  // ---- finished build batches join the sweeps; idle lanes admit new batches
  // With nothing to sweep, a step waits for a build to finish, but at most
  // kServeWaitUs: the caller gets control back to submit new arrivals (which
  // an idle lane can start building at once) and calls step again.
  auto poll_lanes = [&](bool wait) -> mdp_status {
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::microseconds(kServeWaitUs);
    for (;;) {
      bool joined = false, busy = false;
      for (int li = 0; li < kServeLanes; ++li) {
        BuildLane &L = S->lane[li];
        if (!L.solving.empty()) {  // the large lane's solve: keep it fed, retire it when it ends
          if (mdp_status pr = serve_pump_solve(S, L); pr != MDP_OK) return pr;
          const hipError_t q = L.solve_tail ? hipEventQuery(L.solve_ev) : hipErrorNotReady;
          if (q == hipSuccess) {
            serve_solve_retire(S, L);
            joined = true;
          } else if (q == hipErrorNotReady) {
            busy = true;
          } else {
            return hip_fail(S->ctx, q, "serve solve");
          }
          continue;
        }
        if (L.building.empty()) continue;
        if (mdp_status pr = serve_pump(S, L); pr != MDP_OK) return pr;
        if (!L.tail) {
          busy = true;
          continue;
        }
        hipError_t q = hipEventQuery(L.event);
        if (q == hipSuccess) {
          if (li == kServeSolveLane) {
            if (mdp_status pr = serve_solve_start(S, L); pr != MDP_OK) return pr;
          } else {
            serve_join(S, L);
          }
          joined = true;
        } else if (q == hipErrorNotReady) {
          busy = true;
        } else {
          return hip_fail(S->ctx, q, "serve build");
        }
      }
      if (joined || !busy || !wait || std::chrono::steady_clock::now() >= t_end) return MDP_OK;
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  };
  auto admit_idle = [&]() -> mdp_status {
    for (int li = 0; li < kServeLanes; ++li)
      if (S->lane[li].building.empty() && S->lane[li].solving.empty() && !S->queue.empty()) {
        mdp_status r2 = serve_admit(S, li);
        if (r2 != MDP_OK) return r2;
      }
    return MDP_OK;
  };
  auto n_act = [&]() {
    return (int32_t)(S->queue.size() + S->n_building() + S->n_solving() + S->running.size() + S->to_retire.size() +
                     S->retiring.size());
  };
  // ---- completed retirements: records, memory back to the pool
  auto finish_retire = [&]() {
    const mdp_vi_stats *hf = S->h_fstat.as<mdp_vi_stats>();
    const double *vstart = S->h_vstart.as<double>();
    for (size_t i = 0; i < S->retiring.size(); ++i) {
      ServeReq *r = S->retiring[i];
      r->res.sweeps = hf[i].sweeps;
      r->res.residual = hf[i].residual;
      r->res.v_start = vstart[i];
      r->res.status = r->res.build_status != MDP_OK ? r->res.build_status : hf[i].status;
      r->res.done_step = S->step_no;
      S->done.push_back(r->res);
      unreserve(S, r);
      delete r;
    }
    S->retiring.clear();
  };
  // ---- the step in flight has ended: its requests' status, converged ones to retire
  auto finish_step = [&]() {
    const mdp_vi_stats *hv = S->h_vstat.as<mdp_vi_stats>();
    std::vector<ServeReq *> keep;
    for (size_t i = 0; i < S->step_run.size(); ++i) {
      ServeReq *r = S->step_run[i];
      r->res.sweeps = hv[i].sweeps;
      r->res.residual = hv[i].residual;
      if (r->res.build_status != MDP_OK || hv[i].status == MDP_OK || r->sweeps >= r->limit) S->to_retire.push_back(r);
    }
    for (ServeReq *r : S->running)
      if (std::find(S->to_retire.begin(), S->to_retire.end(), r) == S->to_retire.end()) keep.push_back(r);
    S->running.swap(keep);
    S->step_run.clear();
    S->step_inflight = false;
  };
  auto query = [&](hipEvent_t ev, bool &ended) -> mdp_status {
    const hipError_t q = hipEventQuery(ev);
    ended = q == hipSuccess;
    if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(S->ctx, q, "serve step");
    return MDP_OK;
  };
  bool ended = false;
  if ((rc = poll_lanes(false)) != MDP_OK || (rc = admit_idle()) != MDP_OK) return rc;
  if (!S->retiring.empty()) {
    if ((rc = query(S->ret_ev, ended)) != MDP_OK) return rc;
    if (ended) finish_retire();
  }
  if (S->step_inflight) {
    if ((rc = query(S->step_ev, ended)) != MDP_OK) return rc;
    if (ended) finish_step();
  }
  if (S->step_inflight) {  // the device is still on the last step's sweeps: wait for it a little
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::microseconds(kServeWaitUs);
    for (;;) {
      if ((rc = query(S->step_ev, ended)) != MDP_OK) return rc;
      if (ended) {
        finish_step();
        break;
      }
      if ((rc = poll_lanes(false)) != MDP_OK) return rc;
      if (std::chrono::steady_clock::now() >= t_end) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (S->step_inflight) {
      if (n_active) *n_active = n_act();
      return MDP_OK;
    }
  }
  // ---- retire converged requests (and failed builds): finish, policy, the
  // results into the caller's pinned buffers, then ret_ev
  if (!S->to_retire.empty() && S->retiring.empty()) {
    std::vector<ServeReq *> &ret = S->to_retire;
    const int n = (int)ret.size();
    BatchVIDesc *rd = S->h_vret.as<BatchVIDesc>();
    const size_t rwin = vi_descs(ret, rd);
    int64_t *bs = S->h_bsret.as<int64_t>();
    bs[0] = 0;
    for (int i = 0; i < n; ++i) bs[i + 1] = bs[i] + rd[i].P.n_blocks;
    if ((e = hipMemcpyAsync(S->d_vret, rd, sizeof(BatchVIDesc) * n, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(S->d_bs_ret, bs, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_vi_finish_batched(S->d_vret, n, S->d_vstat, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve finish");
    {
      Timed tm(S->ctx, MDP_KERNEL_POLICY, s);
      if ((e = launch_policy_batched(S->d_vret, n, S->d_bs_ret, kBatchViGrid, rwin, s)) != hipSuccess)
        return hip_fail(S->ctx, e, "serve policy");
    }
    double *vstart = S->h_vstart.as<double>();
    for (int i = 0; i < n; ++i) {
      ServeReq *r = ret[i];
      const size_t ns = (size_t)r->z.ns;
      const int64_t s0 = (int64_t)r->p.start_j * r->p.nx + r->p.start_i;
      if ((e = hipMemcpyAsync(&vstart[i], r->v + s0, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (r->h_pi && (e = hipMemcpyAsync(r->h_pi, r->pi, 4 * ns, hipMemcpyDeviceToHost, s)) != hipSuccess) ||
          (r->h_v && (e = hipMemcpyAsync(r->h_v, r->v, 8 * ns, hipMemcpyDeviceToHost, s)) != hipSuccess))
        return hip_fail(S->ctx, e, "serve results");
    }
    if ((e = hipMemcpyAsync(S->h_fstat.p, S->d_vstat, sizeof(mdp_vi_stats) * n, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipEventRecord(S->ret_ev, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve retire");
    S->retiring.swap(S->to_retire);
  }
  if (S->running.empty() && S->n_building() + S->n_solving() > 0) {  // nothing to sweep until a lane ends
    if ((rc = poll_lanes(true)) != MDP_OK || (rc = admit_idle()) != MDP_OK) return rc;
  }
  if (S->running.empty()) {
    if (n_active) *n_active = n_act();
    return MDP_OK;
  }
  // ---- sweeps, shortest remaining work first, without starving the oldest:
  // this step sweeps the built requests whose remaining work (rows times
  // sweeps still to run) is within kServeWorkRatio of the smallest, and the
  // earliest-submitted built request in any case; the others wait (their
  // state is untouched). The step's work is enqueued and the call returns; a
  // later call reads the status once step_ev has completed.
  std::vector<ServeReq *> &run = S->step_run;
  run.clear();
  {
    double wmin = 0.0;
    const ServeReq *oldest = nullptr;
    for (ServeReq *r : S->running) {
      const double w = (double)r->z.rows * (r->limit - r->sweeps);
      if (!oldest || w < wmin) wmin = w;
      if (!oldest || r->seq < oldest->seq) oldest = r;
    }
    for (ServeReq *r : S->running)
      if (r == oldest || (double)r->z.rows * (r->limit - r->sweeps) <= kServeWorkRatio * wmin) run.push_back(r);
  }
  const int n_run = (int)run.size();
  BatchVIDesc *vd = S->h_vrun.as<BatchVIDesc>();
  const size_t win = vi_descs(run, vd);
  if ((e = hipMemcpyAsync(S->d_vrun, vd, sizeof(BatchVIDesc) * n_run, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve solve descriptors");
  for (int i = 0; i < n_run; ++i) {
    ServeReq *r = run[i];
    if (!r->cold) continue;
    if ((e = launch_vi_reset_batched(S->d_vrun + i, 1, s)) != hipSuccess) return hip_fail(S->ctx, e, "serve reset");
    r->cold = false;
  }
  int k = S->cfg.sweeps_per_step;
  for (ServeReq *r : run) k = std::min(k, r->limit - r->sweeps);
  k = std::max(k, 1);
  std::vector<int> behind(n_run);
  for (int i = 0; i < n_run; ++i) behind[i] = run[i]->sweeps;
  std::vector<int64_t> tabs;
  active_block_tables(vd, behind.data(), n_run, k, tabs);
  memcpy(S->h_tables.p, tabs.data(), sizeof(int64_t) * tabs.size());
  if ((e = hipMemcpyAsync(S->d_bs_sweeps, S->h_tables.p, sizeof(int64_t) * tabs.size(), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return hip_fail(S->ctx, e, "serve sweep tables");
  for (int j = 0; j < k; ++j) {
    Timed tm(S->ctx, MDP_KERNEL_VI_SWEEP, s);
    if ((e = launch_vi_sweep_batched(S->d_vrun, n_run, S->d_bs_sweeps + (size_t)j * (n_run + 1), S->d_wg_res,
                                     kBatchViGrid, win, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve sweep");
    if ((e = launch_vi_close_batched(S->d_vrun, n_run, kBatchViGrid, S->d_wg_res, S->cfg.tol, s)) != hipSuccess)
      return hip_fail(S->ctx, e, "serve close");
  }
  for (ServeReq *r : run) r->sweeps += k;
  if ((e = launch_vi_status_batched(S->d_vrun, n_run, S->d_vstat, s)) != hipSuccess ||
      (e = hipMemcpyAsync(S->h_vstat.p, S->d_vstat, sizeof(mdp_vi_stats) * n_run, hipMemcpyDeviceToHost, s)) !=
          hipSuccess ||
      (e = hipEventRecord(S->step_ev, s)) != hipSuccess)
    return hip_fail(S->ctx, e, "serve vi stats");
  S->step_inflight = true;
  if (n_active) *n_active = n_act();
  return MDP_OK;
}

mdp_status mdp_server_poll(mdp_server *S, mdp_served *out, int32_t max_out, int32_t *n_out)
{
  if (!S || !n_out || max_out < 0 || (max_out > 0 && !out)) return MDP_E_INVALID;
  const int n = std::min<int>(max_out, (int)S->done.size());
  for (int i = 0; i < n; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + n);
  *n_out = n;
  return MDP_OK;
}

mdp_status mdp_server_info(mdp_server *S, mdp_server_state *out)
{
  if (!S || !out) return MDP_E_INVALID;
  out->queued = (int32_t)S->queue.size();
  out->in_flight =
      (int32_t)(S->n_building() + S->n_solving() + S->running.size() + S->to_retire.size() + S->retiring.size());
  out->completed = (int32_t)S->done.size();
  out->pad = 0;
  out->pool_used = (int64_t)S->alloc.used();
  out->steps = S->step_no;
  return MDP_OK;
}

mdp_status mdp_server_destroy(mdp_server *S)
{
  if (!S) return MDP_E_INVALID;
  serve_free_all(S);
  return MDP_OK;
}

}  // extern "C"
