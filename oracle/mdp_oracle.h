/*
 * CPU oracle for the stochastic-flow MDP planner: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow reference of what the planner computes, written from the paper
 * (Chowdhury & Subramani, "Optimal Path Planning of Autonomous Marine Vehicles
 * in Stochastic Dynamic Ocean Flows using a GPU-Accelerated Algorithm"):
 *   - transition counts P(s'|s,a) by Monte-Carlo over flow realizations
 *     (Sec. II-A, transition model and cell(); Sec. II-C flow decomposition),
 *   - expected one-step rewards (Eqs. Rsa_time, Rsa_energyConsumption,
 *     Rsa_NetEnergy, with only the scalar field's mean per Sec. III-A),
 *   - optimal values and a greedy policy (Sec. II-B, Bellman equation and
 *     value-iteration update) by finite-horizon backward induction and by
 *     synchronous value iteration, both in double precision.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library. It shares no code with the GPU planner.
 */
#ifndef MDP_ORACLE_H
#define MDP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_problem {
  int32_t nx, ny, nt;          /* spatial grid and number of decision layers  */
  int32_t n_modes, n_real;     /* K DO modes, N_r flow realizations           */
  int32_t n_head, n_speed;     /* N_h headings, N_F speeds                    */
  int32_t sub_hx, sub_hy;      /* neighbouring sub-grid half widths           */
  int32_t start_i, start_j, target_i, target_j;
  int32_t mean_time_varying, mode_time_varying;
  uint32_t mission_mask, flags;
  double dx, dy, dt, f_max;
  double r_term, r_outbound, c_f, c_r;
} ora_problem;

typedef struct ora_env {
  const float *ubar, *vbar;    /* [Tm][ny][nx]                                */
  const float *phiu, *phiv;    /* [Tp][K][ny][nx]                             */
  const float *mu;             /* [nt][K][n_real]                             */
  const float *gbar;           /* [nt+1][ny][nx] or NULL                      */
  const uint8_t *mask;         /* [nt+1][ny][nx] or NULL                      */
} ora_env;

/* Problem flags the oracle reads (bit values of the planner's problem flags). */
#define ORA_FLAG_NEAR_EDGE 1u
#define ORA_FLAG_SWEPT_PATH 2u /* a landing whose straight path from the cell centre
                                  enters an obstacle cell at t+1 is DEAD        */

/* Does the segment from (x0, y0) to (x1, y1) (cell units) meet the interior of
 * cell (a, b), the open square (a, a+1) x (b, b+1)? Exact for the coordinates
 * the planner produces (see the definition). */
int ora_segment_meets_cell(double x0, double y0, double x1, double y1, int a, int b);

/* Action tables: displacement of heading/speed a in cell units and its speed. */
void ora_action_tables(const ora_problem *p, float *hx, float *hy, double *speed);

/* Landing of one sample in FP32 (cell indices) and its near-edge flag. */
void ora_landing(const ora_problem *p, const ora_env *e, int t, int c, int r, int a,
                 int32_t *ip, int32_t *jp, int32_t *near_edge);

/* One row (t, c, a): columns ascending (DEAD = nt*nx*ny, TARGET = DEAD + 1),
 * counts, per-mission expected reward R[3] and expected |reward| A[3].
 * cols/cnts need room for n_real entries. Returns the row's nnz. */
int32_t ora_row(const ora_problem *p, const ora_env *e, int t, int c, int a,
                int32_t *cols, int32_t *cnts, double R[3], double A[3],
                int64_t *n_escape, int64_t *n_near_edge);

/* Every row, in order row = ((t*ny + j)*nx + i)*N_a + a. Writes at most cap
 * entries; returns the total nnz (call again with a larger cap if it exceeds).
 * R and A are [3][rows]; row_near may be NULL, else [rows] near-edge counts. */
int64_t ora_build(const ora_problem *p, const ora_env *e, int64_t *row_ptr, int32_t *col,
                  int32_t *cnt, int64_t cap, double *R, double *A, int32_t *row_near,
                  int64_t *n_escape, int64_t *n_near_edge);

/* ora_build restricted to the decision layers [t0, t1): row_ptr, R, A and
 * row_near hold only those layers' rows (row_ptr[0] = 0), in the same order. */
int64_t ora_build_layers(const ora_problem *p, const ora_env *e, int t0, int t1, int64_t *row_ptr,
                         int32_t *col, int32_t *cnt, int64_t cap, double *R, double *A, int32_t *row_near,
                         int64_t *n_escape, int64_t *n_near_edge);

/* Finite-horizon backward induction, t = nt-1 .. 0. R, A are [rows] for one
 * mission; v, w are [nt*nx*ny]; pi [nt*nx*ny]. A and w may be NULL. */
void ora_backward(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
                  const int32_t *cnt, const double *R, const double *A,
                  double *v, int32_t *pi, double *w);

/* Synchronous value iteration from v (in: v0, out: result). Returns sweeps run;
 * residual history in res[max_sweeps] (may be NULL). */
int32_t ora_jacobi(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
                   const int32_t *cnt, const double *R, double tol, int32_t max_sweeps,
                   double *v, double *res);

/* Q(s, a) for every action of the states listed in s_idx (n of them), from a
 * value vector v: q is [n][N_a]. */
void ora_q(const ora_problem *p, const int64_t *row_ptr, const int32_t *col,
           const int32_t *cnt, const double *R, const double *v,
           const int64_t *s_idx, int64_t n, double *q);

/* Outcome of one rollout (ora_rollout). */
#define ORA_ROLL_ARRIVED 0   /* reached the target                              */
#define ORA_ROLL_OUTBOUND 1  /* a landing left the domain                       */
#define ORA_ROLL_OBSTACLE 2  /* landed on (or started in) an obstacle           */
#define ORA_ROLL_HORIZON 3   /* still travelling after the last decision layer  */

/* Follow the policy pi [nt*nx*ny] from the start cell at t = 0 in every flow
 * realization r (the realization's coefficients mu[t][.][r] at each layer).
 * Per realization: traj [n_real][nt+1] the cell index at each layer (-1 once
 * the path has ended; the target cell at the arrival layer), outcome, the
 * decision steps taken, the realized return of each mission ret [n_real][3]
 * (the one-step rewards of the landings along the path), the energy expended
 * (sum of c_f F^2 dt) and the sum of the speeds used. traj may be NULL. */
void ora_rollout(const ora_problem *p, const ora_env *e, const int32_t *pi, int32_t *traj,
                 int32_t *outcome, int32_t *steps, double *ret, double *energy, double *fsum);

/* Largest |u| and |v| over all synthesised velocities (t, c, r) in FP32. */
void ora_max_speed(const ora_problem *p, const ora_env *e, double *umax, double *vmax);

/* Smallest half widths h with h + 1/2 > (U + F_max) dt/d + 1e-3, per axis. */
void ora_subgrid_auto(const ora_problem *p, const ora_env *e, int32_t *hx, int32_t *hy);

#ifdef __cplusplus
}
#endif
#endif
