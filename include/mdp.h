/*
 * mdp.h -- C ABI of the MI355X stochastic-flow MDP planner (libmdp.so).
 *
 * The planner implements the end-to-end method of Chowdhury & Subramani,
 * "Optimal Path Planning of Autonomous Marine Vehicles in Stochastic Dynamic
 * Ocean Flows using a GPU-Accelerated Algorithm":
 *   mdp_build          -- Alg. 1 / Alg. 2: Monte-Carlo transition counts over
 *                         flow realizations binned in a neighbouring sub-grid
 *                         (Sec. III-B, III-C) and the expected one-step reward
 *                         of each mission (Eqs. Rsa_time, Rsa_energyConsumption,
 *                         Rsa_NetEnergy with the mean scalar field, Sec. III-A);
 *   mdp_value_iterate  -- value iteration v_{k+1} = max_a sum P [r + v_k]
 *                         (Sec. II-B, Sec. III-D);
 *   mdp_policy         -- greedy policy pi = argmax_a sum P [r + v] (Sec. II-B).
 *
 * Conventions shared by every call
 *   - Grid: nx * ny cells of size dx * dy, cell (i, j) = [i dx, (i+1) dx) x
 *     [j dy, (j+1) dy); a state is (t, i, j) for decision layers t = 0..nt-1,
 *     positioned at the cell centre (Sec. II-A).
 *   - State index s = (t*ny + j)*nx + i, N_s = nt*nx*ny. Two absorbing sinks
 *     follow the states: DEAD = N_s (obstacle, outside the domain, or beyond
 *     the horizon) and TARGET = N_s + 1; both have value 0.
 *   - Actions: a = jf*n_head + h with heading angle 2*pi*h/n_head
 *     (counter-clockwise from east) and speed f_max*(jf+1)/n_speed.
 *   - Row index of (s, a) is s*N_a + a, N_a = n_head*n_speed.
 *   - Every device pointer is owned by the caller; the library never frees
 *     caller memory and allocates no device memory inside these calls.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream). Argument errors are returned synchronously; errors found
 *     by the device are reported in the stats struct once the stream reaches
 *     the end of the call.
 *   - No call throws; every call returns an mdp_status.
 *   - A context may be used by one host thread at a time. Calls that share a
 *     scratch buffer must be ordered on one stream.
 */
#ifndef MDP_H
#define MDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdp_status;
#define MDP_OK 0
#define MDP_E_INVALID 1       /* bad argument, shape or pointer                    */
#define MDP_E_CAPACITY 2      /* nnz_capacity too small; stats.nnz holds the need  */
#define MDP_E_SUBGRID 3       /* a landing left the sub-grid; stats.n_escape > 0   */
#define MDP_E_HIP 4           /* a HIP runtime call failed                          */
#define MDP_E_NOT_CONVERGED 5 /* value iteration stopped at max_sweeps              */
#define MDP_E_SCRATCH 6       /* scratch buffer smaller than mdp_build_query says   */

#define MDP_MISSION_TIME 0       /* R = -dt                                      */
#define MDP_MISSION_ENERGY 1     /* R = -c_f F^2 dt                              */
#define MDP_MISSION_NET_ENERGY 2 /* R = E[-c_f F^2 + c_r (g(s) + g(s'))/2] dt    */

#define MDP_FLAG_NEAR_EDGE 1u /* count samples within 1e-6 (physical) of an edge */
/* Swept-path obstacle test (the path reading of Alg. 2's "obstacle between s
 * and s'"): a landing is DEAD (r_outbound) when the straight step from the
 * source cell centre to the landing point enters the interior of a cell, other
 * than the source cell, that is an obstacle at t+1; without the flag only the
 * landing cell is checked. Used by mdp_build, mdp_build_from and mdp_rollout;
 * batches and servers refuse it (MDP_E_INVALID). A row may then hold one entry
 * more than its sub-grid has cells: nnz_upper = rows * min(N_sg + 1, n_real). */
#define MDP_FLAG_SWEPT_PATH 2u

#define MDP_MAX_ACTIONS 64
#define MDP_MAX_MODES 16

/* Problem statement: Alg. 1's prob_type, prob_params and grid_params. */
typedef struct mdp_problem {
  int32_t nx, ny, nt;        /* grid cells per axis and decision layers          */
  int32_t n_modes, n_real;   /* K flow modes (<= 16), N_r realizations (<= 65535) */
  int32_t n_head, n_speed;   /* headings and speeds, N_a = product <= 64          */
  int32_t sub_hx, sub_hy;    /* sub-grid half widths; N_sg = (2hx+1)(2hy+1)       */
  int32_t start_i, start_j;  /* start cell (reporting only)                       */
  int32_t target_i, target_j;/* target cell                                       */
  int32_t mean_time_varying; /* 0: ubar/vbar hold one layer, 1: nt layers         */
  int32_t mode_time_varying; /* 0: phiu/phiv hold one layer, 1: nt layers         */
  uint32_t mission_mask;     /* bit m set: build the reward of mission m          */
  uint32_t flags;            /* MDP_FLAG_*                                        */
  double dx, dy, dt, f_max;  /* cell sizes, time step, top agent speed            */
  double r_term, r_outbound; /* arrival bonus, failure reward (Table I)           */
  double c_f, c_r;           /* energy e(F) = c_f F^2; harvest coefficient c_r    */
} mdp_problem;

/* Reduced-order environment (Sec. II-C, Alg. 1 REQUIRE), device pointers,
 * row-major, fp32 unless noted:
 *   ubar, vbar  [Tm][ny][nx]     DO mean, Tm = nt if mean_time_varying else 1
 *   phiu, phiv  [Tp][K][ny][nx]  DO modes, Tp = nt if mode_time_varying else 1
 *   mu          [nt][K][n_real]  DO coefficients, realization index fastest
 *   gbar        [nt+1][ny][nx]   mean scalar field; required for NET_ENERGY
 *   mask        uint8 [nt+1][ny][nx]  obstacle mask (nonzero = blocked), or NULL */
typedef struct mdp_env {
  const float *ubar, *vbar;
  const float *phiu, *phiv;
  const float *mu;
  const float *gbar;
  const uint8_t *mask;
} mdp_env;

/* Sparse model in CSR, device pointers. Rows are ordered (t, j, i, a); the
 * columns of a row are ascending (transient states of layer t+1, then DEAD,
 * then TARGET); P(s'|s,a) = cnt / n_real.
 *   row_ptr  int64  [N_s*N_a + 1]
 *   col      int32  [nnz_capacity]
 *   cnt      uint16 [nnz_capacity]    realizations landing in col
 *   reward   fp32   [n_missions][N_s*N_a]  one block per set bit of
 *                   mission_mask, in ascending mission order
 *   ent      uint32 [nnz_capacity], or NULL: the same nonzeros packed for
 *                   value iteration, (window index << 16) | cnt, where the
 *                   window index is the column's position in the grid rows of
 *                   layer t+1 that the sweep stages for the row's block of
 *                   cells, and 0xFFFF marks DEAD and TARGET. mdp_build and
 *                   mdp_build_from fill it when it is not NULL and the
 *                   problem's window fits (rows of (2 sub_hy + 2) grid rows of
 *                   nx cells in 16 KB; otherwise it is left untouched), and
 *                   mdp_value_iterate_missions then reads it instead of col
 *                   and cnt: 4 bytes per nonzero instead of 6, same results
 *                   bit for bit. Only a model built by mdp_build /
 *                   mdp_build_from with this ent may be solved with it.
 *   roff     uint16 [N_s*N_a], NULL exactly when ent is NULL: each row's
 *                   first entry relative to the first entry of its sweep
 *                   block (B = min(512 / N_a, N_x N_y) consecutive cells of
 *                   one layer, all their actions), written with ent; the
 *                   packed sweep reads it instead of row_ptr (2 bytes per row
 *                   instead of 8). Packing also needs every block's entries
 *                   to fit 16 bits: B * N_a * max_row <= 65535, max_row =
 *                   min(sub-grid cells, plus one with MDP_FLAG_SWEPT_PATH,
 *                   n_real); otherwise ent and roff are left untouched and
 *                   unused. ent and roff are both NULL or both set
 *                   (MDP_E_INVALID otherwise).                             */
typedef struct mdp_model {
  int64_t *row_ptr;
  int32_t *col;
  uint16_t *cnt;
  float *reward;
  int64_t nnz_capacity;
  uint32_t *ent;
  uint16_t *roff;
} mdp_model;

/* Sizes of a problem (host-only arithmetic, no device work). */
typedef struct mdp_sizes {
  int64_t n_states;        /* N_s                                              */
  int64_t n_actions;       /* N_a                                              */
  int64_t n_rows;          /* N_s * N_a                                        */
  int64_t n_sg;            /* sub-grid cells                                   */
  int64_t nnz_upper;       /* n_rows * min(N_sg, n_real): never exceeded        */
  int64_t n_missions;      /* set bits of mission_mask                         */
  int64_t scratch_bytes;   /* scratch needed by mdp_build / mdp_value_iterate  */
  int64_t env_bytes;       /* bytes of the environment arrays                  */
  int64_t layers_per_slab; /* decision layers handled per build pass           */
} mdp_sizes;

typedef struct mdp_build_stats {
  int64_t samples;     /* (state, action, realization) landings computed       */
  int64_t nnz;         /* nonzeros of the model (also when above capacity)     */
  int64_t n_escape;    /* landings outside the sub-grid (must be 0)            */
  int64_t n_near_edge; /* landings within 1e-6 of a cell edge; -1 if not asked */
  int32_t status;      /* MDP_OK, MDP_E_CAPACITY or MDP_E_SUBGRID              */
  int32_t n_slabs;     /* build passes                                         */
} mdp_build_stats;

typedef struct mdp_vi_stats {
  int32_t sweeps;   /* synchronous sweeps run                                  */
  int32_t status;   /* MDP_OK or MDP_E_NOT_CONVERGED                           */
  double residual;  /* max_s |v_k(s) - v_{k-1}(s)| of the last sweep           */
} mdp_vi_stats;

typedef struct mdp_ctx mdp_ctx;

/* Context bound to one HIP device: small internal scratch, the last error
 * text and the per-kernel timing records. */
mdp_status mdp_ctx_create(int32_t device, mdp_ctx **out);
mdp_status mdp_ctx_destroy(mdp_ctx *ctx);

/* Static description of a status code. */
const char *mdp_status_str(mdp_status s);

/* Text of the last error recorded on this context ("" if none). */
const char *mdp_last_error(const mdp_ctx *ctx);

/* Sizes of every buffer a caller allocates for problem p (Alg. 1's
 * allocations, done once by the caller instead of per (t, a)). */
mdp_status mdp_build_query(const mdp_problem *p, mdp_sizes *out);

/* Neighbouring sub-grid dimension (Alg. 1, "compute dimension"; Sec. III-B):
 * the smallest hx, hy with h + 1/2 > (U + f_max) dt/d + 1e-3, U the largest
 * |u| (|v|) over every synthesised velocity (t, cell, realization) in fp32.
 * Runs on the device and waits for it (synchronous). p->sub_hx/hy are ignored. */
mdp_status mdp_subgrid_auto(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env,
                            int32_t *hx, int32_t *hy, void *stream);

/* Build the sparse model (Alg. 1 with Alg. 2's per-sample work).
 *   scratch      device buffer of at least mdp_sizes.scratch_bytes (enough for
 *                any launch shape the context may have tuned)
 *   stats        host memory written when the stream reaches the end of the
 *                call (pinned memory keeps the call asynchronous)
 * Landing cells are decided in fp32 with one fused multiply-add per mode term
 * and per position update, so counts are reproducible bit for bit. */
mdp_status mdp_build(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env,
                     const mdp_model *model, void *scratch, size_t scratch_bytes,
                     mdp_build_stats *stats, void *stream);

/* Incremental re-planning (the paper's in-mission updates of the forecast,
 * Sec. I and Sec. V): rebuild, in place, the rows of the decision layers
 * [t0, nt) of a model that holds a complete build of the same problem, after
 * the environment changed from layer t0 on (new coefficients mu[t >= t0], new
 * mean or modes at t >= t0, new mask or scalar field at layers > t0). The rows
 * of layers < t0 and their entries are kept; the rebuilt entries follow them,
 * so the result equals mdp_build on the new environment bit for bit as long
 * as the rows of layers < t0 did not change (a layer-(t0-1) row reads the mask
 * and scalar field of layer t0: rebuild from t0 - 1 when those changed).
 * stats->samples counts the rebuilt layers' landings and stats->nnz the whole
 * model's nonzeros (MDP_E_CAPACITY above nnz_capacity). Same scratch as
 * mdp_build. */
mdp_status mdp_build_from(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const mdp_model *model,
                          int32_t t0, void *scratch, size_t scratch_bytes, mdp_build_stats *stats, void *stream);

/* Wait for `stream` to reach the end of an mdp_build and return the device
 * status it reported (Alg. 1 ENSURE: the model is complete only once this is
 * MDP_OK). `stats` is the host struct passed to that mdp_build. Returns
 * MDP_OK, MDP_E_CAPACITY (stats->nnz is the capacity needed), MDP_E_SUBGRID
 * (stats->n_escape landings left the sub-grid; the model is not valid), or
 * MDP_E_HIP if the stream reported an error; the last error text names the
 * figures. */
mdp_status mdp_build_sync(mdp_ctx *ctx, const mdp_build_stats *stats, void *stream);

/* Synchronous (Jacobi) value iteration on the model of mission `mission`
 * (Sec. II-B update rule), from the values in d_v (v0; zeros for a cold start)
 * until max_s |v_k - v_{k-1}| < tol or max_sweeps sweeps. Values are fp64,
 * [N_s]; the result is left in d_v. Sums of each row are taken in a fixed
 * order, so the layered model reaches a residual of exactly 0 after at most
 * nt + 1 sweeps. */
mdp_status mdp_value_iterate(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model,
                             int32_t mission, double tol, int32_t max_sweeps, double *d_v,
                             void *scratch, size_t scratch_bytes, mdp_vi_stats *stats,
                             void *stream);

/* Bytes of the library's static device scratch used by
 * mdp_value_iterate_noalloc (one copy per GPU, held until the process ends):
 * the sweep state, device stats, the second fp64 value buffer [N_s] and the
 * per-workgroup residuals, i.e. problems of up to about 9.4 million states. */
#define MDP_NOALLOC_SCRATCH_BYTES ((size_t)72 << 20)

/* mdp_value_iterate without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The call allocates nothing: its scratch
 * is the library's static per-GPU array of MDP_NOALLOC_SCRATCH_BYTES, whose
 * address the context looked up at mdp_ctx_create; it runs the same kernels
 * as mdp_value_iterate and gives the same d_v and stats bit for bit. The
 * caller still owns d_v (v0 in, result out, fp64 [N_s]) and the host stats.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call initialises what it reads before reading it):
 * calls that overlap in time on one GPU (on different streams, or from
 * several host threads or contexts) race and must be ordered on one stream.
 * Sweeps are not recorded by mdp_ctx_profile. Errors: MDP_E_SCRATCH when the
 * problem needs more than MDP_NOALLOC_SCRATCH_BYTES (the text gives the
 * figure), MDP_E_INVALID as mdp_value_iterate, MDP_E_HIP if the context could
 * not look up the array. */
mdp_status mdp_value_iterate_noalloc(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                                     double tol, int32_t max_sweeps, double *d_v, mdp_vi_stats *stats, void *stream);

/* Value iteration of the decision layers [t_first, nt) only (re-planning from
 * layer t_first on: every transition goes from layer t to t + 1 or to a sink,
 * so those layers depend on nothing earlier). The values of layers < t_first
 * in d_v are left as they are; those of layers >= t_first end up equal to
 * mdp_value_iterate's from the same v0, bit for bit, after at most
 * nt - t_first + 1 sweeps (stats count these sweeps and their residuals, over
 * the layers solved). Same scratch as mdp_value_iterate. */
mdp_status mdp_value_iterate_layers(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model, int32_t mission,
                                    int32_t t_first, double tol, int32_t max_sweeps, double *d_v, void *scratch,
                                    size_t scratch_bytes, mdp_vi_stats *stats, void *stream);

/* mdp_value_iterate for n_missions (1..3) distinct missions of one model in
 * one solve (Sec. II-B update rule per mission). Each sweep reads the model's
 * transition entries once for all of them; every mission keeps its own values,
 * residual, sweep count and stopping test, so d_v[i] and stats[i] are exactly
 * what mdp_value_iterate gives for missions[i] from the same v0 (bit for bit).
 * d_v: n_missions device pointers, each fp64 [N_s] (v0 in, result out);
 * stats: n_missions host structs, written when the stream reaches the end of
 * the solve. scratch: device memory of at least n_missions times
 * mdp_build_query's scratch_bytes. Errors: MDP_E_INVALID (a mission not built,
 * repeated missions or value buffers, host pointers), MDP_E_SCRATCH. */
mdp_status mdp_value_iterate_missions(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model,
                                      int32_t n_missions, const int32_t *missions, double tol,
                                      int32_t max_sweeps, double *const *d_v, void *scratch,
                                      size_t scratch_bytes, mdp_vi_stats *stats, void *stream);

/* Greedy policy (Sec. II-B): d_pi[s] = the lowest action index attaining
 * max_a R(s,a) + sum_s' P(s'|s,a) v(s'), for every state. d_v fp64 [N_s],
 * d_pi int32 [N_s]. */
mdp_status mdp_policy(mdp_ctx *ctx, const mdp_problem *p, const mdp_model *model,
                      int32_t mission, const double *d_v, int32_t *d_pi, void *stream);

/* ------------------------------------------------------------------ rollouts
 * The policy applied to every realization of the stochastic flow (Sec. IV:
 * each optimal policy is followed through the ensemble of flow fields, giving
 * the distribution of paths, the expected travel time and energy).
 * In realization r the agent starts in (start_i, start_j) at t = 0; at layer t
 * in cell c it takes action pi[t][c] and lands where realization r's flow
 * puts it, computed with the FP32 operations of mdp_build (so every landing is
 * a sample of the transition model). The landing ends the path outside the
 * domain or on an obstacle at t+1 (reward r_outbound), on the target (base +
 * r_term, arrived) or beyond the horizon (r_outbound); otherwise the path goes
 * on with reward base (Table I, Eqs. Rsa_time / Rsa_energyConsumption /
 * Rsa_NetEnergy with the mean scalar field). A path starting on the target has
 * arrived after 0 steps (return 0); one starting in an obstacle ends at once
 * with return r_outbound. */
#define MDP_ROLL_ARRIVED 0
#define MDP_ROLL_OUTBOUND 1
#define MDP_ROLL_OBSTACLE 2
#define MDP_ROLL_HORIZON 3
typedef struct mdp_rollout_path {
  int32_t outcome;  /* MDP_ROLL_*                                                */
  int32_t steps;    /* decisions taken                                           */
  double ret[3];    /* realized return of missions time, energy, net energy      */
  double energy;    /* energy expended, sum of c_f F^2 dt over the steps         */
  double fsum;      /* sum of the speeds of the actions taken                    */
} mdp_rollout_path;
typedef struct mdp_rollout_stats {
  int64_t n_real, n_arrived, n_outbound, n_obstacle, n_horizon;
  double p_reach;                 /* n_arrived / n_real                        */
  double mean_time_arrived;       /* mean steps * dt over the arrived paths    */
  double mean_energy_arrived;     /* mean energy expended over arrived paths   */
  double mean_net_energy_arrived; /* mean net energy consumed (expended minus
                                     harvested from the mean scalar field)     */
  double mean_speed_arrived;      /* speed sum / steps over the arrived paths  */
  double mean_return[3];          /* mean realized return over all paths       */
} mdp_rollout_stats;
/* Device scratch bytes of mdp_rollout for problem p (host only). */
mdp_status mdp_rollout_query(const mdp_problem *p, size_t *scratch_bytes);
/* Roll the policy d_pi (int32 [nt][ny][nx], device; entries outside [0, N_a)
 * are read as action 0) out in all n_real realizations of env (device
 * pointers as for mdp_build; gbar may be NULL, then the net-energy return has
 * no harvest term). d_traj: int32 [nt+1][n_real] device, layer-major (the
 * cell index at each layer, the target cell at the arrival layer, -1 after the
 * end), or NULL. d_paths: [n_real] device, or NULL (then kept in scratch).
 * stats: host, written when the stream reaches the end of the call. Errors:
 * MDP_E_INVALID (pointers, problem), MDP_E_SCRATCH. */
mdp_status mdp_rollout(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, const int32_t *d_pi,
                       int32_t *d_traj, mdp_rollout_path *d_paths, void *scratch, size_t scratch_bytes,
                       mdp_rollout_stats *stats, void *stream);

/* ------------------------------------------------------------------ batches
 * Many independent problems built and solved together (not in the paper: the
 * batched form of the calls above). mdp_batch_create takes every pointer up
 * front and uploads one device descriptor table, so build and solve only
 * enqueue kernels and can be captured into a HIP graph:
 *   - the build is one persistent launch over a work list of (problem, layer,
 *     cell tile) items sorted by cost, each item's entries staged in a
 *     bump-allocated pool of pool_entries 8-byte entries (0: 4 per row of the
 *     batch), then a per-problem scan and one copy launch into each CSR;
 *   - the solve runs one sweep launch per iteration over the state blocks of
 *     every problem that has not converged (per-problem residual, done flag and
 *     sweep count), then the greedy policy of each problem.
 * Every problem's model, values and policy equal those of mdp_build /
 * mdp_value_iterate / mdp_policy on it alone, bit for bit.
 * Ownership: models, values (fp64 [N_s]; every solve starts from v0 = 0),
 * policies and scratch are caller-owned device buffers; the batch owns only its
 * descriptor table. Device-side errors appear in mdp_batch_stats:
 * MDP_E_CAPACITY (model too small), MDP_E_SCRATCH (staging pool too small),
 * MDP_E_SUBGRID. At most 1024 problems. */
typedef struct mdp_batch mdp_batch;
mdp_status mdp_batch_query(int32_t n, const mdp_problem *probs, int64_t pool_entries, size_t *scratch_bytes);
mdp_status mdp_batch_create(mdp_ctx *ctx, int32_t n, const mdp_problem *probs, const mdp_env *envs,
                            const mdp_model *models, const int32_t *missions, double *const *d_v,
                            int32_t *const *d_pi, int64_t pool_entries, void *scratch, size_t scratch_bytes,
                            mdp_batch **out);
mdp_status mdp_batch_build(mdp_batch *b, void *stream);
mdp_status mdp_batch_solve(mdp_batch *b, double tol, int32_t max_sweeps, void *stream);
/* Copies the per-problem stats to the host (waits for the device). Either
 * pointer may be NULL. */
mdp_status mdp_batch_stats(mdp_batch *b, mdp_build_stats *build_stats, mdp_vi_stats *vi_stats);
/* Record build + solve on `stream` (not the null stream) into a HIP graph
 * owned by the batch; mdp_batch_replay launches it. */
mdp_status mdp_batch_capture(mdp_batch *b, double tol, int32_t max_sweeps, void *stream);
mdp_status mdp_batch_replay(mdp_batch *b, void *stream);
mdp_status mdp_batch_destroy(mdp_batch *b);

/* ------------------------------------------------------------------ serving
 * Continuous batching of planning requests (not in the paper). Requests queue
 * in arrival order; each mdp_server_step
 *   1. admits queued requests while a slot is free and the pool holds the
 *      request's footprint (mdp_server_footprint: model with the worst-case
 *      nonzeros rows * min(N_sg, n_real), values, policy, and its share of the
 *      build scratch); small and large builds have a lane each (a stream, one
 *      build batch at a time), requests are admitted in arrival order within
 *      their size class, and a batch holds builds within a factor 4 in cost;
 *   2. builds every newly admitted request in one batched build, split into
 *      short launches that the other lane and the sweeps interleave with, and,
 *      once it has finished, gives the unused part of the worst-case
 *      reservation back to the pool;
 *   3. runs up to sweeps_per_step synchronous sweeps over every admitted
 *      request in one launch per sweep (requests joined at different sweeps);
 *   4. retires each request that converged (or reached its sweep limit):
 *      greedy policy, copies of the policy / values into the caller's host
 *      buffers, completion record, pool space freed.
 * Each request's model, values and policy equal those of mdp_build /
 * mdp_value_iterate / mdp_policy on it alone, bit for bit. Only the requested
 * mission's reward is built. The step waits for the device before returning.
 * Ownership: the pool is a caller-owned device range; env arrays and h_pi /
 * h_v (host, int32 / fp64 [N_s], may be NULL; pinned memory keeps the copies
 * asynchronous) must stay valid until the request's completion is polled. */
typedef struct mdp_server mdp_server;
typedef struct mdp_server_config {
  int32_t max_inflight;    /* requests admitted at once, 1..1024                */
  int32_t sweeps_per_step; /* most sweeps a step enqueues, 1..256               */
  int32_t max_sweeps;      /* a request retires unconverged after this many     */
  int32_t build_share;     /* percent of the resident workgroups a build batch
                              may hold (1..100; 0 = 100); the rest keeps
                              sweeping the admitted requests meanwhile          */
  double tol;              /* residual below which a request has converged      */
  double chunk_cost;       /* build work per launch of a served build, in
                              landings (each plus a quarter per mode term per
                              action); 0 = 6e9 (about 2 ms on an MI355X)        */
  double large_cost;       /* requests whose build cost (same unit) exceeds this
                              build on the large-request lane; 0 = 3e10         */
} mdp_server_config;
typedef struct mdp_served {
  int64_t tag;                   /* the submitter's tag                         */
  int64_t nnz, samples;          /* model size and landings computed            */
  int64_t admit_step, done_step; /* step numbers (1-based) of admission / retirement */
  double residual;               /* last sweep's residual                       */
  double v_start;                /* value of (t = 0, start cell)                */
  int32_t status;                /* MDP_OK, a build error, or MDP_E_NOT_CONVERGED */
  int32_t build_status;
  int32_t sweeps, pad;
} mdp_served;
typedef struct mdp_server_state {
  int32_t queued, in_flight, completed, pad;
  int64_t pool_used, steps;
} mdp_server_state;
/* Pool bytes a request of problem p holds at admission. */
mdp_status mdp_server_footprint(const mdp_problem *p, size_t *bytes);
mdp_status mdp_server_create(mdp_ctx *ctx, const mdp_server_config *cfg, void *pool, size_t pool_bytes,
                             mdp_server **out);
/* Queue a request (no device work). MDP_E_CAPACITY if it can never fit the pool. */
mdp_status mdp_server_submit(mdp_server *srv, const mdp_problem *p, const mdp_env *env, int32_t mission,
                             int32_t *h_pi, double *h_v, int64_t tag);
/* One scheduler iteration on `stream` (the same stream on every call);
 * n_active = queued + admitted afterwards. It admits queued requests into idle
 * build lanes, retires the requests the last completed step found converged
 * (finish, policy, copies into their pinned buffers) and enqueues the sweeps
 * of the built requests chosen this step (shortest remaining work first, the
 * earliest-submitted one always), then returns without waiting for them; a
 * later call reads their status. While the previous step's sweeps run, or
 * with nothing built to sweep, a call waits at most about 0.5 ms, so callers
 * loop on it while n_active > 0 and submit new arrivals between calls. */
mdp_status mdp_server_step(mdp_server *srv, void *stream, int32_t *n_active);
/* Move up to max_out completion records (oldest first) into out. */
mdp_status mdp_server_poll(mdp_server *srv, mdp_served *out, int32_t max_out, int32_t *n_out);
mdp_status mdp_server_info(mdp_server *srv, mdp_server_state *out);
mdp_status mdp_server_destroy(mdp_server *srv);

/* ------------------------------------------------------------------ tuning
 * The build kernel's launch shape (lanes owning a (cell, action) row: 256, 128
 * or 64, which fixes the cell tile; realizations per chunk: 64, 128 or 256;
 * 16- or 32-bit LDS counters) changes only speed: every shape gives the same
 * model bit for bit. A context keeps one shape per shape class of problem
 * (actions, sub-grid, mode bound, near-edge counting, log2 of realizations and
 * cells); mdp_build, batches and servers created on the context use it, others
 * use the default shape.
 * mdp_autotune times every shape that fits p on a sample of p's first layers
 * (16384 cell tiles of the default shape, or all layers; the caller's env is
 * read, scratch holds the sample's model and build scratch, size from
 * mdp_autotune_query), waits for the device,
 * records the fastest for p's class and reports all timings.
 * mdp_ctx_set_plan sets a class's shape directly (row_lanes = 0: default). */
#define MDP_MAX_TUNE 18
typedef struct mdp_tune_report {
  int32_t n_candidates;      /* shapes timed                                  */
  int32_t best;              /* index of the fastest                          */
  int32_t sample_layers;     /* layers of the timed sample                    */
  int32_t default_shape;     /* index of the shape used without tuning        */
  int32_t row_lanes[MDP_MAX_TUNE], rch[MDP_MAX_TUNE], pack16[MDP_MAX_TUNE];
  double ms[MDP_MAX_TUNE];   /* best of two timed builds of the sample        */
} mdp_tune_report;
mdp_status mdp_autotune_query(const mdp_problem *p, size_t *scratch_bytes);
mdp_status mdp_autotune(mdp_ctx *ctx, const mdp_problem *p, const mdp_env *env, void *scratch,
                        size_t scratch_bytes, mdp_tune_report *out, void *stream);
mdp_status mdp_ctx_set_plan(mdp_ctx *ctx, const mdp_problem *p, int32_t row_lanes, int32_t rch,
                            int32_t pack16);

/* Per-kernel timing. While enabled, HIP events are recorded on the caller's
 * stream around every launch of the kernels below; mdp_ctx_profile_read waits
 * for the recorded events and returns the launch count and summed duration.
 * Enabling (enable = 1) clears earlier records; disabling keeps them. */
#define MDP_KERNEL_BUILD 0    /* histogram + compaction pass of mdp_build  */
#define MDP_KERNEL_VI_SWEEP 1 /* one synchronous sweep of mdp_value_iterate */
#define MDP_KERNEL_POLICY 2   /* mdp_policy                                 */
#define MDP_KERNEL_COPY 3     /* staging-to-CSR copy of mdp_build           */
#define MDP_N_KERNELS 4
mdp_status mdp_ctx_profile(mdp_ctx *ctx, int32_t enable);
mdp_status mdp_ctx_profile_read(mdp_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* MDP_H */
