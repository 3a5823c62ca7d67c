// Host side of the C ABI declared in include/mdp.h: argument checks, launch
// planning (tile shape, realization chunk, LDS size, layers per pass), scratch
// layout, and the enqueue order of the build / value-iteration / policy kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "mdp_internal.h"

using namespace mdpk;

struct mdp_ctx {
  int device;
  unsigned int *d_small;  // 256 bytes of device memory for synchronous helpers
  char err[512];
  // per-kernel timing (only while profiling is enabled)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[MDP_N_KERNELS];
  size_t ev_used[MDP_N_KERNELS] = {};
};

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kStageBudget = size_t(4) << 30;  // staging bytes per build pass
constexpr size_t kLdsLimit = 160 * 1024;

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

const char *make_plan(const mdp_problem *p, Plan &pl)
{
  if (const char *e = check_problem(p)) return e;
  pl.na = p->n_head * p->n_speed;
  pl.nc = p->nx * p->ny;
  pl.W = 2 * p->sub_hx + 1;
  pl.nsg = pl.W * (2 * p->sub_hy + 1);
  pl.rows = (int64_t)p->nt * pl.nc * pl.na;
  pl.pack16 = true;  // n_real <= 65535, so two 16-bit counters fit a word
  pl.kmax = p->n_modes <= 4 ? 4 : (p->n_modes <= 8 ? 8 : 16);
  const size_t fixed_lds = 2 * kMaxA * sizeof(float) + 16 * sizeof(uint32_t);
  bool ok = false;
  for (int rl = kBlock; rl >= 64 && !ok; rl /= 2) {
    if (rl < pl.na) break;
    const int hw = pl.pack16 ? rl / 2 : rl;
    const int cells = std::min(rl / pl.na, 32);
    const int rch = cells <= 8 ? 256 : (cells <= 16 ? 128 : 64);
    const size_t lds = (size_t)pl.nsg * hw * 4 + (size_t)cells * (2 * rch + 4) * 4 + fixed_lds;
    if (lds <= kLdsLimit) {
      pl.row_lanes = rl;
      pl.hw = hw;
      pl.cells_per_tile = cells;
      pl.rch = rch;
      pl.lds = lds;
      ok = true;
    }
  }
  if (!ok) return "sub-grid too large for the LDS histogram";
  pl.tiles_per_layer = (pl.nc + pl.cells_per_tile - 1) / pl.cells_per_tile;
  pl.wg_cap = (int64_t)pl.cells_per_tile * pl.na * std::min(pl.nsg, p->n_real);
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
  pl.vi_bytes = align_up(sizeof(VIState)) + align_up(sizeof(mdp_vi_stats)) + align_up((size_t)ns * 8);
  return nullptr;
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
void action_tables(const mdp_problem *p, float *hx, float *hy)
{
  const double kPi = 3.14159265358979323846;
  for (int jf = 0; jf < p->n_speed; ++jf) {
    const double F = p->f_max * (double)(jf + 1) / (double)p->n_speed;
    for (int h = 0; h < p->n_head; ++h) {
      const double th = 2.0 * kPi * (double)h / (double)p->n_head;
      const int a = jf * p->n_head + h;
      hx[a] = (float)(F * cos(th) * p->dt / p->dx);
      hy[a] = (float)(F * sin(th) * p->dt / p->dy);
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
  out->nnz_upper = pl.rows * (int64_t)std::min(pl.nsg, p->n_real);
  out->n_missions = popcount3(p->mission_mask);
  out->scratch_bytes = (int64_t)std::max(pl.build_bytes, pl.vi_bytes);
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

mdp_status mdp_build(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                     void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream)
{
  if (!ctx) return MDP_E_INVALID;
  Plan pl;
  if (const char *e = make_plan(p, pl)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (const char *e = check_env(p, env)) {
    set_err(ctx, "%s", e);
    return MDP_E_INVALID;
  }
  if (!model || !is_device_ptr(model->row_ptr) || !is_device_ptr(model->reward) ||
      (model->nnz_capacity > 0 && (!is_device_ptr(model->col) || !is_device_ptr(model->cnt)))) {
    set_err(ctx, "model buffers must be device pointers");
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
  if ((e = launch_build_init(st, s)) != hipSuccess) return hip_fail(ctx, e, "init");
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
    for (int t0 = 0; t0 < p->nt; t0 += pl.layers_per_slab, ++n_slabs) {
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
        if ((e = launch_build_slab(P, S, pl.kmax, pl.pack16, near, pl.lds, s)) != hipSuccess)
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
  if ((e = launch_build_finalize(st, model->nnz_capacity, n_slabs, near ? 1 : 0, s)) != hipSuccess)
    return hip_fail(ctx, e, "finalize");
  if ((e = hipMemcpyAsync(stats, &st->out, sizeof(mdp_build_stats), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(ctx, e, "stats copy");
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
      !is_device_ptr(model->reward)) {
    set_err(ctx, "model buffers must be device pointers");
    return MDP_E_INVALID;
  }
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
  V.states_per_wg = kBlock / pl.na;
  V.n_blocks = (V.ns + V.states_per_wg - 1) / V.states_per_wg;
  V.n_wg = (int)std::min<int64_t>(V.n_blocks, 2048);
  V.inv_nr = 1.0 / (double)p->n_real;
  return MDP_OK;
}

mdp_status mdp_value_iterate(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                             double tol, int32_t max_sweeps, double *d_v, void *scratch, size_t scratch_bytes,
                             mdp_vi_stats *stats, void *stream)
{
  Plan pl;
  VIParams V;
  mdp_status rc = vi_setup(ctx, p, model, mission, pl, V);
  if (rc != MDP_OK) return rc;
  if (!is_device_ptr(d_v) || !stats || max_sweeps < 0) {
    set_err(ctx, "d_v must be a device pointer, stats non-NULL, max_sweeps >= 0");
    return MDP_E_INVALID;
  }
  if (!is_device_ptr(scratch) || scratch_bytes < pl.vi_bytes) {
    set_err(ctx, "scratch needs %zu device bytes", pl.vi_bytes);
    return MDP_E_SCRATCH;
  }
  char *sc = (char *)scratch;
  V.st = (VIState *)sc;
  mdp_vi_stats *dstats = (mdp_vi_stats *)(sc + align_up(sizeof(VIState)));
  double *v_alt = (double *)(sc + align_up(sizeof(VIState)) + align_up(sizeof(mdp_vi_stats)));
  V.tol = tol;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = launch_vi_init(V.st, s)) != hipSuccess) return hip_fail(ctx, e, "vi init");
  // The model is layered in time, so a positive tolerance is met after at most
  // nt + 1 sweeps (the last one has residual exactly 0): no host polling.
  int n = max_sweeps;
  if (tol > 0.0) n = std::min(n, p->nt + 1);
  for (int k = 0; k < n; ++k) {
    const double *vin = (k & 1) ? v_alt : d_v;
    double *vout = (k & 1) ? d_v : v_alt;
    Timed tm(ctx, MDP_KERNEL_VI_SWEEP, s);
    if ((e = launch_vi_sweep(V, vin, vout, k & 1, s)) != hipSuccess) return hip_fail(ctx, e, "vi sweep");
  }
  if ((e = launch_vi_finish(V, d_v, v_alt, dstats, s)) != hipSuccess) return hip_fail(ctx, e, "vi finish");
  if ((e = hipMemcpyAsync(stats, dstats, sizeof(mdp_vi_stats), hipMemcpyDeviceToHost, s)) != hipSuccess)
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

}  // extern "C"
