// Policy rollouts through the flow-realization ensemble (the use the paper
// makes of each optimal policy in Sec. IV: the policy applied to every
// realization of the stochastic flow, giving the distribution of paths, the
// expected travel time and the expected energy).
//
// One lane follows one realization r: at layer t in cell c it takes action
// pi(t, c), synthesises that realization's flow at (t, c) from the
// coefficients mu[t][.][r] (realization fastest, so a wave's coefficient loads
// are one coalesced 256-byte read per mode), and lands with exactly the FP32
// operations of the model build (one fma per mode term, px = fma(u, dt/dx,
// i + 1/2), X = px + Hx[a], floor), so a path's landings are samples of the
// transition model bit for bit. The landing is classified with the model's
// rules and its one-step reward is added to the realized return of every
// mission. Trajectories are stored layer-major ([t][r]) so that the lanes of a
// wave write one contiguous line per step.
//
// The ensemble statistics (outcome counts, P(reach), means over the arrived
// paths, mean returns) come from a one-workgroup reduction in a fixed order,
// so repeated calls give the same bits.
#include "mdp_internal.h"

namespace mdpk {

__global__ __launch_bounds__(kBlock) void k_rollout(const RollParams P)
{
  __shared__ float hx_s[kMaxA], hy_s[kMaxA];
  __shared__ double sp_s[kMaxA];
  for (int a = threadIdx.x; a < kMaxA; a += kBlock) {
    hx_s[a] = P.tab.hx[a];
    hy_s[a] = P.tab.hy[a];
    sp_s[a] = P.speed[a];
  }
  __syncthreads();
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= P.nr) return;
  const int nx = P.nx, ny = P.ny, nt = P.nt, nc = P.nc;
  int32_t *tr = P.traj;
  int i = P.si, j = P.sj, n = 0, out = MDP_ROLL_HORIZON;
  double R0 = 0.0, R1 = 0.0, R2 = 0.0, E = 0.0, Fs = 0.0;
  if (tr) tr[r] = j * nx + i;
  int t = 0;
  for (; t < nt; ++t) {
    const int c = j * nx + i;
    if (i == P.ti && j == P.tj) {  // only a start on the target
      out = MDP_ROLL_ARRIVED;
      break;
    }
    if (P.mask != nullptr && P.mask[(size_t)t * nc + c] != 0) {  // only a start inside an obstacle
      R0 += P.r_out;
      R1 += P.r_out;
      R2 += P.r_out;
      out = MDP_ROLL_OBSTACLE;
      break;
    }
    const int a = P.pi[(size_t)t * nc + c];
    const size_t tm = (size_t)P.mean_tstride * t, tp = (size_t)P.mode_tstride * t;
    float u = P.ubar[tm + c];
    float v = P.vbar[tm + c];
    const float *mu_t = P.mu + (size_t)t * P.K * P.nr + r;
    for (int k = 0; k < P.K; ++k) {
      const float m = mu_t[(size_t)k * P.nr];
      u = __builtin_fmaf(m, P.phiu[tp + (size_t)k * nc + c], u);
      v = __builtin_fmaf(m, P.phiv[tp + (size_t)k * nc + c], v);
    }
    const float px = __builtin_fmaf(u, P.lam_x, (float)i + 0.5f);
    const float py = __builtin_fmaf(v, P.lam_y, (float)j + 0.5f);
    const int ai = (unsigned)a < (unsigned)P.na ? a : 0;  // a policy entry outside [0, N_a) is read as 0
    const float X = px + hx_s[ai];
    const float Y = py + hy_s[ai];
    const int ip = (int)floorf(X), jp = (int)floorf(Y);
    const double F = sp_s[ai], e_a = P.c_f * F * F;
    ++n;
    E += e_a * P.dt;
    Fs += F;
    if (ip < 0 || ip >= nx || jp < 0 || jp >= ny) {
      R0 += P.r_out;
      R1 += P.r_out;
      R2 += P.r_out;
      out = MDP_ROLL_OUTBOUND;
      break;
    }
    const int cp = jp * nx + ip;
    if (P.mask != nullptr && (P.mask[(size_t)(t + 1) * nc + cp] != 0 ||
                              (P.swept && swept_blocked(P.mask + (size_t)(t + 1) * nc, nx, ny, i, j, ip, jp, X, Y)))) {
      R0 += P.r_out;
      R1 += P.r_out;
      R2 += P.r_out;
      out = MDP_ROLL_OBSTACLE;
      break;
    }
    const double g_s = P.gbar ? (double)P.gbar[(size_t)t * nc + c] : 0.0;
    const double g_sp = P.gbar ? (double)P.gbar[(size_t)(t + 1) * nc + cp] : 0.0;
    const double b0 = -P.dt, b1 = -e_a * P.dt, b2 = (-e_a + 0.5 * P.c_r * g_s + 0.5 * P.c_r * g_sp) * P.dt;
    if (ip == P.ti && jp == P.tj) {
      R0 += b0 + P.r_term;
      R1 += b1 + P.r_term;
      R2 += b2 + P.r_term;
      if (tr) tr[(size_t)(t + 1) * P.nr + r] = cp;
      ++t;
      out = MDP_ROLL_ARRIVED;
      break;
    }
    if (t + 1 == nt) {
      R0 += P.r_out;
      R1 += P.r_out;
      R2 += P.r_out;
      out = MDP_ROLL_HORIZON;
      break;
    }
    R0 += b0;
    R1 += b1;
    R2 += b2;
    i = ip;
    j = jp;
    if (tr) tr[(size_t)(t + 1) * P.nr + r] = cp;
  }
  if (tr)  // layers after the end of the path
    for (int k = t + 1; k <= nt; ++k) tr[(size_t)k * P.nr + r] = -1;
  mdp_rollout_path o;
  o.outcome = out;
  o.steps = n;
  o.ret[0] = R0;
  o.ret[1] = R1;
  o.ret[2] = R2;
  o.energy = E;
  o.fsum = Fs;
  P.paths[r] = o;
}

constexpr int kRollRed = 256;  // threads of the statistics reduction

// Sums of the paths in a fixed order: thread k takes paths k, k + kRollRed,
// ..., then a fixed pairwise tree over the threads.
__global__ __launch_bounds__(kRollRed) void k_rollout_stats(const mdp_rollout_path *paths, int nr, double dt,
                                                            double r_term, mdp_rollout_stats *out)
{
  // outcome counts (4); over arrived paths: steps, energy, net energy, speed
  // sum (4); returns of the three missions over all paths (3)
  constexpr int NQ = 11;
  __shared__ double sh[NQ][kRollRed];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int r = threadIdx.x; r < nr; r += kRollRed) {
    const mdp_rollout_path &o = paths[r];
    const bool arr = o.outcome == MDP_ROLL_ARRIVED;
    acc[0] += arr ? 1.0 : 0.0;
    acc[1] += o.outcome == MDP_ROLL_OUTBOUND ? 1.0 : 0.0;
    acc[2] += o.outcome == MDP_ROLL_OBSTACLE ? 1.0 : 0.0;
    acc[3] += o.outcome == MDP_ROLL_HORIZON ? 1.0 : 0.0;
    if (arr) {
      acc[4] += (double)o.steps;
      acc[5] += o.energy;
      acc[6] += r_term - o.ret[2];  // net energy consumed by an arrived path
      acc[7] += o.fsum;
    }
    acc[8] += o.ret[0];
    acc[9] += o.ret[1];
    acc[10] += o.ret[2];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kRollRed / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int q = 0; q < NQ; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mdp_rollout_stats s;
    const double na = sh[0][0];
    s.n_real = nr;
    s.n_arrived = (int64_t)na;
    s.n_outbound = (int64_t)sh[1][0];
    s.n_obstacle = (int64_t)sh[2][0];
    s.n_horizon = (int64_t)sh[3][0];
    s.p_reach = nr > 0 ? na / (double)nr : 0.0;
    s.mean_time_arrived = na > 0 ? sh[4][0] * dt / na : 0.0;
    s.mean_energy_arrived = na > 0 ? sh[5][0] / na : 0.0;
    s.mean_net_energy_arrived = na > 0 ? sh[6][0] / na : 0.0;
    s.mean_speed_arrived = sh[4][0] > 0 ? sh[7][0] / sh[4][0] : 0.0;
    for (int m = 0; m < 3; ++m) s.mean_return[m] = nr > 0 ? sh[8 + m][0] / (double)nr : 0.0;
    *out = s;
  }
}

hipError_t launch_rollout(const RollParams &P, mdp_rollout_stats *dev_stats, hipStream_t s)
{
  if (P.nr > 0) {
    hipLaunchKernelGGL(k_rollout, dim3((P.nr + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rollout_stats, dim3(1), dim3(kRollRed), 0, s, (const mdp_rollout_path *)P.paths, P.nr, P.dt,
                     P.r_term, dev_stats);
  return hipGetLastError();
}

}  // namespace mdpk
