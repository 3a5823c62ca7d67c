/*
 * CPU oracle for the stochastic-flow MDP planner: TEST INFRASTRUCTURE ONLY.
 * See mdp_oracle.h for the scope. Compile with -O2 -ffp-contract=off and
 * without fast-math: the landing cell is decided in FP32 in the operation order
 * stated at ora_landing, and nothing else may reorder or contract it.
 *
 * Everything here is deliberately the plainest form of each definition:
 * every sample is binned over the full domain (no neighbouring sub-grid),
 * counts come from sorting the landing columns, rewards are averaged in double
 * precision in ascending realization order, and values come from backward
 * induction over the layered time grid.
 */
#include "mdp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORA_PI 3.14159265358979323846
#define ORA_MAX_ACTIONS 256

/* Heading h of N_h is the angle 2*pi*h/N_h counter-clockwise from east; speed
 * j of N_F is F_max*(j+1)/N_F; action a = j*N_h + h (Sec. II-A: N_h headings in
 * [0, 2pi) times N_F speeds in (0, F_max]). The displacement a*dt in cell units
 * is evaluated in double and rounded to FP32 once. A heading along an axis
 * (a whole number of quarter turns) has the exact direction components 0 and
 * +-1, so it moves along that axis only. */
void ora_action_tables(const ora_problem *p, float *hx, float *hy, double *speed)
{
  for (int jf = 0; jf < p->n_speed; ++jf) {
    double F = p->f_max * (double)(jf + 1) / (double)p->n_speed;
    for (int h = 0; h < p->n_head; ++h) {
      double c, s;
      if ((4 * h) % p->n_head == 0) {
        const int quarter = (4 * h) / p->n_head;  /* 0..3 */
        c = quarter == 0 ? 1.0 : (quarter == 2 ? -1.0 : 0.0);
        s = quarter == 1 ? 1.0 : (quarter == 3 ? -1.0 : 0.0);
      } else {
        double th = 2.0 * ORA_PI * (double)h / (double)p->n_head;
        c = cos(th);
        s = sin(th);
      }
      int a = jf * p->n_head + h;
      if (hx) hx[a] = (float)(F * c * p->dt / p->dx);
      if (hy) hy[a] = (float)(F * s * p->dt / p->dy);
      if (speed) speed[a] = F;
    }
  }
}

static int n_actions(const ora_problem *p) { return p->n_head * p->n_speed; }

/* Flow at state (t, cell c) in realization r: mean plus sum over modes of
 * coefficient times mode (Sec. II-C decomposition), accumulated in ascending
 * mode order with one fused multiply-add per term, in FP32. */
static void ora_velocity(const ora_problem *p, const ora_env *e, int t, int c, int r,
                         float *u_out, float *v_out)
{
  const size_t nc = (size_t)p->nx * p->ny;
  const size_t tm = p->mean_time_varying ? (size_t)t : 0;
  const size_t tp = p->mode_time_varying ? (size_t)t : 0;
  float u = e->ubar[tm * nc + c];
  float v = e->vbar[tm * nc + c];
  for (int k = 0; k < p->n_modes; ++k) {
    float m = e->mu[((size_t)t * p->n_modes + k) * p->n_real + r];
    u = fmaf(m, e->phiu[(tp * p->n_modes + k) * nc + c], u);
    v = fmaf(m, e->phiv[(tp * p->n_modes + k) * nc + c], v);
  }
  *u_out = u;
  *v_out = v;
}

/* The kinematic step x' = x + (v + a) dt and s' = cell(x', t + dt) of Sec. II-A,
 * in cell units with cell (i, j) = [i, i+1) x [j, j+1) and the state at the
 * cell centre (i + 1/2, j + 1/2). FP32 order:
 *   px = fma(u, dt/dx, i + 1/2);  X = px + Hx[a];  i' = floor(X)   (same in y)
 * A sample is near an edge when X or Y lies within 1e-6 (physical units) of
 * an integer. */
static void landing_xy(const ora_problem *p, const ora_env *e, const float *hx, const float *hy,
                       int t, int c, int r, int a, int32_t *ip, int32_t *jp, int32_t *near_edge,
                       float *Xo, float *Yo)
{
  const int i = c % p->nx, j = c / p->nx;
  const float lam_x = (float)(p->dt / p->dx), lam_y = (float)(p->dt / p->dy);
  const float eps_x = (float)(1e-6 / p->dx), eps_y = (float)(1e-6 / p->dy);
  float u, v;
  ora_velocity(p, e, t, c, r, &u, &v);
  float px = fmaf(u, lam_x, (float)i + 0.5f);
  float py = fmaf(v, lam_y, (float)j + 0.5f);
  float X = px + hx[a];
  float Y = py + hy[a];
  *ip = (int32_t)floorf(X);
  *jp = (int32_t)floorf(Y);
  *near_edge = (fabsf(X - rintf(X)) < eps_x) || (fabsf(Y - rintf(Y)) < eps_y);
  if (Xo) *Xo = X;
  if (Yo) *Yo = Y;
}

static void landing(const ora_problem *p, const ora_env *e, const float *hx, const float *hy,
                    int t, int c, int r, int a, int32_t *ip, int32_t *jp, int32_t *near_edge)
{
  landing_xy(p, e, hx, hy, t, c, r, a, ip, jp, near_edge, NULL, NULL);
}

void ora_landing(const ora_problem *p, const ora_env *e, int t, int c, int r, int a,
                 int32_t *ip, int32_t *jp, int32_t *near_edge)
{
  float hx[ORA_MAX_ACTIONS], hy[ORA_MAX_ACTIONS];
  ora_action_tables(p, hx, hy, NULL);
  landing(p, e, hx, hy, t, c, r, a, ip, jp, near_edge);
}

/* Separating-axis test of a closed segment against an open unit square: they
 * meet iff their projections overlap on the x axis, on the y axis and on the
 * segment's normal. With P0 = (i + 1/2, j + 1/2) and P1 = (X, Y) from FP32
 * landings (coordinates below 2^24 in magnitude with 24-bit mantissas), every
 * difference and product below is exact in double precision, so the test is
 * exact and its outcome does not depend on the evaluation order. */
int ora_segment_meets_cell(double x0, double y0, double x1, double y1, int a, int b)
{
  const double lx = x0 < x1 ? x0 : x1, hx = x0 < x1 ? x1 : x0;
  const double ly = y0 < y1 ? y0 : y1, hy = y0 < y1 ? y1 : y0;
  if (!(lx < (double)a + 1.0 && hx > (double)a)) return 0;
  if (!(ly < (double)b + 1.0 && hy > (double)b)) return 0;
  const double dx = x1 - x0, dy = y1 - y0;
  double fmin = 0.0, fmax = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double cx = (double)(a + (k & 1)), cy = (double)(b + (k >> 1));
    const double f = dx * (cy - y0) - dy * (cx - x0); /* side of the corner w.r.t. the line */
    if (k == 0 || f < fmin) fmin = f;
    if (k == 0 || f > fmax) fmax = f;
  }
  return fmin < 0.0 && fmax > 0.0;
}

/* Swept-path reading of the obstacle test of Alg. 2: the straight path of the
 * step from the source cell centre to the landing point crosses an obstacle
 * cell at t+1 other than the source cell. */
static int swept_blocked(const ora_problem *p, const ora_env *e, int t, int i, int j, float X, float Y)
{
  if (!(p->flags & ORA_FLAG_SWEPT_PATH) || !e->mask) return 0;
  const int nx = p->nx, ny = p->ny;
  const double x0 = (double)i + 0.5, y0 = (double)j + 0.5, x1 = (double)X, y1 = (double)Y;
  const int a0 = (int)floor(x0 < x1 ? x0 : x1), a1 = (int)floor(x0 < x1 ? x1 : x0);
  const int b0 = (int)floor(y0 < y1 ? y0 : y1), b1 = (int)floor(y0 < y1 ? y1 : y0);
  for (int b = b0; b <= b1; ++b)
    for (int a = a0; a <= a1; ++a) {
      if ((a == i && b == j) || a < 0 || a >= nx || b < 0 || b >= ny) continue;
      if (!e->mask[(size_t)(t + 1) * nx * ny + (size_t)b * nx + a]) continue;
      if (ora_segment_meets_cell(x0, y0, x1, y1, a, b)) return 1;
    }
  return 0;
}

static int cmp_i32(const void *x, const void *y)
{
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

/* One (t, c, a) row.
 *  - The target cell is absorbing: every realization goes to TARGET, R = 0.
 *  - An obstacle cell at t sends every realization to DEAD with r_outbound.
 *  - Otherwise each realization lands somewhere; in this order, a landing
 *    outside the domain, on an obstacle at t+1, on the target, or past the
 *    horizon (t+1 = nt) is DEAD, TARGET, DEAD; anything else is state (t+1, c').
 * Per-sample reward (Table I terms, Eqs. Rsa_time / Rsa_energyConsumption /
 * Rsa_NetEnergy with the mean scalar field of Sec. III-A):
 *    base_time   = -dt
 *    base_energy = -c_f F^2 dt
 *    base_net    = (-c_f F^2 + c_r gbar(s)/2 + c_r gbar(s')/2) dt
 *    DEAD: r = r_outbound (replaces the base); TARGET: r = base + r_term.
 * R is the sample mean over realizations, summed in ascending order. */
int32_t ora_row(const ora_problem *p, const ora_env *e, int t, int c, int a,
                int32_t *cols, int32_t *cnts, double R[3], double A[3],
                int64_t *n_escape, int64_t *n_near_edge)
{
  const int nx = p->nx, ny = p->ny, nt = p->nt;
  const int nc = nx * ny;
  const int32_t ns = nt * nc;
  const int32_t DEAD = ns, TARGET = ns + 1;
  const int i = c % nx, j = c / nx;
  const int nr = p->n_real;

  if (i == p->target_i && j == p->target_j) {
    cols[0] = TARGET;
    cnts[0] = nr;
    for (int m = 0; m < 3; ++m) R[m] = A[m] = 0.0;
    return 1;
  }
  if (e->mask && e->mask[(size_t)t * nc + c]) {
    cols[0] = DEAD;
    cnts[0] = nr;
    for (int m = 0; m < 3; ++m) {
      R[m] = p->r_outbound;
      A[m] = fabs(p->r_outbound);
    }
    return 1;
  }

  double speed[ORA_MAX_ACTIONS];
  float hx[ORA_MAX_ACTIONS], hy[ORA_MAX_ACTIONS];
  ora_action_tables(p, hx, hy, speed);
  const double F = speed[a];
  const double e_a = p->c_f * F * F;
  const double g_s = e->gbar ? (double)e->gbar[(size_t)t * nc + c] : 0.0;

  int32_t *land = (int32_t *)malloc(sizeof(int32_t) * (size_t)nr);
  double sum[3] = {0, 0, 0}, asum[3] = {0, 0, 0};
  for (int r = 0; r < nr; ++r) {
    int32_t ip, jp, ne;
    float X, Y;
    landing_xy(p, e, hx, hy, t, c, r, a, &ip, &jp, &ne, &X, &Y);
    if (ne) ++*n_near_edge;
    if (abs(ip - i) > p->sub_hx || abs(jp - j) > p->sub_hy) ++*n_escape;

    int32_t col;
    double rr[3];
    if (ip < 0 || ip >= nx || jp < 0 || jp >= ny || swept_blocked(p, e, t, i, j, X, Y)) {
      col = DEAD;
      rr[0] = rr[1] = rr[2] = p->r_outbound;
    } else {
      const int cp = jp * nx + ip;
      const double g_sp = e->gbar ? (double)e->gbar[(size_t)(t + 1) * nc + cp] : 0.0;
      const double base[3] = {
          -p->dt,
          -e_a * p->dt,
          (-e_a + 0.5 * p->c_r * g_s + 0.5 * p->c_r * g_sp) * p->dt,
      };
      if (e->mask && e->mask[(size_t)(t + 1) * nc + cp]) {
        col = DEAD;
        rr[0] = rr[1] = rr[2] = p->r_outbound;
      } else if (ip == p->target_i && jp == p->target_j) {
        col = TARGET;
        for (int m = 0; m < 3; ++m) rr[m] = base[m] + p->r_term;
      } else if (t + 1 == nt) {
        col = DEAD;
        rr[0] = rr[1] = rr[2] = p->r_outbound;
      } else {
        col = (t + 1) * nc + cp;
        for (int m = 0; m < 3; ++m) rr[m] = base[m];
      }
    }
    for (int m = 0; m < 3; ++m) {
      sum[m] += rr[m];
      asum[m] += fabs(rr[m]);
    }
    land[r] = col;
  }
  for (int m = 0; m < 3; ++m) {
    R[m] = sum[m] / (double)nr;
    A[m] = asum[m] / (double)nr;
  }

  /* P(s'|s,a) = (number of realizations landing in s') / N_r */
  qsort(land, (size_t)nr, sizeof(int32_t), cmp_i32);
  int32_t n = 0;
  for (int r = 0; r < nr; ++r) {
    if (n > 0 && cols[n - 1] == land[r]) {
      ++cnts[n - 1];
    } else {
      cols[n] = land[r];
      cnts[n] = 1;
      ++n;
    }
  }
  free(land);
  return n;
}

int64_t ora_build_layers(const ora_problem *p, const ora_env *e, int t0, int t1, int64_t *row_ptr,
                         int32_t *col, int32_t *cnt, int64_t cap, double *R, double *A, int32_t *row_near,
                         int64_t *n_escape, int64_t *n_near_edge)
{
  const int nc = p->nx * p->ny, na = n_actions(p);
  const int64_t rows = (int64_t)(t1 - t0) * nc * na;
  int32_t *tc = (int32_t *)malloc(sizeof(int32_t) * (size_t)p->n_real);
  int32_t *tn = (int32_t *)malloc(sizeof(int32_t) * (size_t)p->n_real);
  int64_t nnz = 0;
  row_ptr[0] = 0;
  *n_escape = 0;
  *n_near_edge = 0;
  for (int t = t0; t < t1; ++t)
    for (int c = 0; c < nc; ++c)
      for (int a = 0; a < na; ++a) {
        const int64_t row = ((int64_t)(t - t0) * nc + c) * na + a;
        double Rr[3], Ar[3];
        int64_t near_before = *n_near_edge;
        int32_t n = ora_row(p, e, t, c, a, tc, tn, Rr, Ar, n_escape, n_near_edge);
        for (int32_t k = 0; k < n; ++k, ++nnz)
          if (nnz < cap) {
            col[nnz] = tc[k];
            cnt[nnz] = tn[k];
          }
        row_ptr[row + 1] = nnz;
        for (int m = 0; m < 3; ++m) {
          if (R) R[m * rows + row] = Rr[m];
          if (A) A[m * rows + row] = Ar[m];
        }
        if (row_near) row_near[row] = (int32_t)(*n_near_edge - near_before);
      }
  free(tc);
  free(tn);
  return nnz;
}

int64_t ora_build(const ora_problem *p, const ora_env *e, int64_t *row_ptr, int32_t *col,
                  int32_t *cnt, int64_t cap, double *R, double *A, int32_t *row_near,
                  int64_t *n_escape, int64_t *n_near_edge)
{
  return ora_build_layers(p, e, 0, p->nt, row_ptr, col, cnt, cap, R, A, row_near, n_escape, n_near_edge);
}

/* Q(s, a) = R(s, a) + sum over transient s' of P(s'|s,a) v(s'); both sinks
 * (DEAD, TARGET) carry value 0. */
static double q_value(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *cnt, const double *R, const double *v, int64_t row)
{
  const int32_t ns = p->nt * p->nx * p->ny;
  double q = R[row];
  for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k)
    if (col[k] < ns) q += ((double)cnt[k] / (double)p->n_real) * v[col[k]];
  return q;
}

void ora_backward(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
                  const int32_t *cnt, const double *R, const double *A,
                  double *v, int32_t *pi, double *w)
{
  const int nc = p->nx * p->ny, na = n_actions(p);
  const int32_t ns = p->nt * nc;
  for (int t = p->nt - 1; t >= 0; --t)
    for (int c = 0; c < nc; ++c) {
      const int64_t s = (int64_t)t * nc + c;
      double best = -INFINITY;
      int32_t besta = 0;
      for (int a = 0; a < na; ++a) {
        double q = q_value(p, row_ptr, col, cnt, R, v, s * na + a);
        if (q > best) { /* first maximiser wins ties */
          best = q;
          besta = a;
        }
      }
      v[s] = best;
      pi[s] = besta;
      if (w) {
        const int64_t row = s * na + besta;
        double ws = A ? A[row] : 0.0;
        for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k)
          if (col[k] < ns) ws += ((double)cnt[k] / (double)p->n_real) * w[col[k]];
        w[s] = ws;
      }
    }
}

int32_t ora_jacobi(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
                   const int32_t *cnt, const double *R, double tol, int32_t max_sweeps,
                   double *v, double *res)
{
  const int na = n_actions(p);
  const int64_t ns = (int64_t)p->nt * p->nx * p->ny;
  double *vn = (double *)malloc(sizeof(double) * (size_t)ns);
  int32_t k = 0;
  while (k < max_sweeps) {
    double rk = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
      double best = -INFINITY;
      for (int a = 0; a < na; ++a) {
        double q = q_value(p, row_ptr, col, cnt, R, v, s * na + a);
        if (q > best) best = q;
      }
      vn[s] = best;
      double d = fabs(best - v[s]);
      if (d > rk) rk = d;
    }
    memcpy(v, vn, sizeof(double) * (size_t)ns);
    if (res) res[k] = rk;
    ++k;
    if (rk < tol) break;
  }
  free(vn);
  return k;
}

void ora_q(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
           const int32_t *cnt, const double *R, const double *v,
           const int64_t *s_idx, int64_t n, double *q)
{
  const int na = n_actions(p);
  for (int64_t k = 0; k < n; ++k)
    for (int a = 0; a < na; ++a)
      q[k * na + a] = q_value(p, row_ptr, col, cnt, R, v, s_idx[k] * na + a);
}

/* Rollout of a policy through the ensemble (Sec. IV applies each optimal
 * policy to every realization of the flow and reports the resulting
 * trajectories, expected travel time and energy). In realization r the agent
 * at layer t in cell c takes action pi(t, c) and lands where the kinematic
 * step of that realization puts it (the same landing as a sample of the
 * transition model); the landing is classified with the rules of ora_row, and
 * its one-step reward is added to the realized return of each mission:
 *   outside the domain or on an obstacle at t+1: r_outbound, the path ends;
 *   the target: base + r_term, the path ends (arrived);
 *   beyond the horizon (t+1 = nt): r_outbound, the path ends;
 *   otherwise base, and the path continues from (t+1, c').
 * A path that starts on the target has arrived after 0 steps with return 0; one
 * that starts in an obstacle ends at once with return r_outbound (the fixed
 * rows of those states). */
void ora_rollout(const ora_problem *p, const ora_env *e, const int32_t *pi, int32_t *traj,
                 int32_t *outcome, int32_t *steps, double *ret, double *energy, double *fsum)
{
  const int nx = p->nx, ny = p->ny, nt = p->nt;
  const int nc = nx * ny;
  double speed[ORA_MAX_ACTIONS];
  float hx[ORA_MAX_ACTIONS], hy[ORA_MAX_ACTIONS];
  ora_action_tables(p, hx, hy, speed);
  for (int r = 0; r < p->n_real; ++r) {
    int32_t *tr = traj ? traj + (size_t)r * (nt + 1) : NULL;
    double R[3] = {0.0, 0.0, 0.0}, E = 0.0, Fs = 0.0;
    int i = p->start_i, j = p->start_j, n = 0, out = ORA_ROLL_HORIZON;
    int t = 0;
    if (tr)
      for (int k = 0; k <= nt; ++k) tr[k] = -1;
    if (tr) tr[0] = j * nx + i;
    for (t = 0; t < nt; ++t) {
      const int c = j * nx + i;
      if (i == p->target_i && j == p->target_j) {
        out = ORA_ROLL_ARRIVED;
        break;
      }
      if (e->mask && e->mask[(size_t)t * nc + c]) {
        for (int m = 0; m < 3; ++m) R[m] += p->r_outbound;
        out = ORA_ROLL_OBSTACLE;
        break;
      }
      const int a = pi[(size_t)t * nc + c];
      int32_t ip, jp, ne;
      float X, Y;
      landing_xy(p, e, hx, hy, t, c, r, a, &ip, &jp, &ne, &X, &Y);
      const double F = speed[a], e_a = p->c_f * F * F;
      ++n;
      E += e_a * p->dt;
      Fs += F;
      if (ip < 0 || ip >= nx || jp < 0 || jp >= ny) {
        for (int m = 0; m < 3; ++m) R[m] += p->r_outbound;
        out = ORA_ROLL_OUTBOUND;
        break;
      }
      const int cp = jp * nx + ip;
      if ((e->mask && e->mask[(size_t)(t + 1) * nc + cp]) || swept_blocked(p, e, t, i, j, X, Y)) {
        for (int m = 0; m < 3; ++m) R[m] += p->r_outbound;
        out = ORA_ROLL_OBSTACLE;
        break;
      }
      const double g_s = e->gbar ? (double)e->gbar[(size_t)t * nc + c] : 0.0;
      const double g_sp = e->gbar ? (double)e->gbar[(size_t)(t + 1) * nc + cp] : 0.0;
      const double base[3] = {-p->dt, -e_a * p->dt, (-e_a + 0.5 * p->c_r * g_s + 0.5 * p->c_r * g_sp) * p->dt};
      if (ip == p->target_i && jp == p->target_j) {
        for (int m = 0; m < 3; ++m) R[m] += base[m] + p->r_term;
        if (tr) tr[t + 1] = cp;
        out = ORA_ROLL_ARRIVED;
        break;
      }
      if (t + 1 == nt) {
        for (int m = 0; m < 3; ++m) R[m] += p->r_outbound;
        out = ORA_ROLL_HORIZON;
        break;
      }
      for (int m = 0; m < 3; ++m) R[m] += base[m];
      i = ip;
      j = jp;
      if (tr) tr[t + 1] = cp;
    }
    outcome[r] = out;
    steps[r] = n;
    for (int m = 0; m < 3; ++m) ret[(size_t)r * 3 + m] = R[m];
    energy[r] = E;
    fsum[r] = Fs;
  }
}

void ora_max_speed(const ora_problem *p, const ora_env *e, double *umax, double *vmax)
{
  const int nc = p->nx * p->ny;
  float mu_ = 0.0f, mv = 0.0f;
  for (int t = 0; t < p->nt; ++t)
    for (int c = 0; c < nc; ++c)
      for (int r = 0; r < p->n_real; ++r) {
        float u, v;
        ora_velocity(p, e, t, c, r, &u, &v);
        if (fabsf(u) > mu_) mu_ = fabsf(u);
        if (fabsf(v) > mv) mv = fabsf(v);
      }
  *umax = mu_;
  *vmax = mv;
}

/* Sub-grid dimension (Alg. 1, "compute dimension for neighbouring sub-grid"):
 * the component-wise maximum flow speed plus the agent's top speed, times
 * dt/dx, plus a 1e-3 cell buffer, must stay below h + 1/2. */
static int32_t half_width(double U, double fmax, double lam)
{
  double z = (U + fmax) * lam + 1e-3;
  int32_t h = (int32_t)floor(z - 0.5) + 1;
  return h < 0 ? 0 : h;
}

void ora_subgrid_auto(const ora_problem *p, const ora_env *e, int32_t *hx, int32_t *hy)
{
  double U, V;
  ora_max_speed(p, e, &U, &V);
  *hx = half_width(U, p->f_max, p->dt / p->dx);
  *hy = half_width(V, p->f_max, p->dt / p->dy);
}
