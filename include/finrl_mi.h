/*
 * finrl_mi.h -- C ABI of the MI355X (gfx950) massively parallel trading-environment rollout.
 *
 * The library implements the simulation ("producer") phase of the training loop the paper
 * describes in Section 3.2: N vectorised stock-trading sub-environments (Section 4.2) whose
 * actions come from a K-actor ensemble (Section 5.2.1), with the samples written as
 * T x N x D device tensors (Section 4.3).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device buffers owned by the caller (for example the data_ptr of a
 *     torch tensor on the current GPU).  Pointers named h_* are host memory.  The library never
 *     allocates device memory: the caller sizes workspaces with the *_workspace_bytes queries
 *     and keeps every buffer alive for as long as a handle that refers to it.
 *   - Work is enqueued on the stream given at creation (environments) or per call (ensemble_act)
 *     and the call returns without synchronising the host, except where stated.
 *   - External layouts are row-major with the last index fastest: actions [N][D], states
 *     [N][S] with S = (I+2)*D+1, trajectories [T][N][...] (Section 4.3).
 *   - Errors: arguments are validated before anything is enqueued; an invalid argument returns
 *     FM_ERR_INVALID, a call that does not fit the environment's current day returns
 *     FM_ERR_STATE, a launch or device failure returns FM_ERR_DEVICE, and a size the kernels do
 *     not support returns FM_ERR_UNSUPPORTED.  Nothing aborts and nothing throws across the ABI;
 *     fm_last_error() describes the most recent failure on the calling thread.
 */
#ifndef FINRL_MI_H
#define FINRL_MI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fm_status {
  FM_OK = 0,
  FM_ERR_INVALID = 1,
  FM_ERR_STATE = 2,
  FM_ERR_DEVICE = 3,
  FM_ERR_UNSUPPORTED = 4
} fm_status;

typedef enum fm_dtype { FM_F32 = 0, FM_BF16 = 1 } fm_dtype;

typedef enum fm_path {
  FM_PATH_PLAIN = 0,  /* per-step launches: ensemble MLP, then noise + trade + reward + state */
  FM_PATH_FUSED = 1   /* one persistent launch that loops over the steps (bfloat16 ensembles) */
} fm_path;

/* Environment parameters.  The MDP is that of Section 3.1: state [b, p, h, f], an action is a
 * change of holdings, reward v_{t+1} - v_t with v_t = b_t + p_t^T h_t. */
typedef struct fm_env_config {
  int32_t n_envs;          /* N sub-environments, >= 1 */
  int32_t n_stocks;        /* D assets, 1..128 */
  int32_t n_ind;           /* I indicators per asset, 0..16 */
  int32_t n_days;          /* T steps; the market arrays hold T+1 days */
  int32_t hmax;            /* shares per unit action, 1..2^20 */
  double init_cash;        /* b_0 >= 0 */
  double cost_rate;        /* proportional transaction cost c in [0, 1) */
  double reward_scale;     /* r_t = (v_{t+1} - v_t) * reward_scale */
  float cash_obs_scale;    /* state entries: fl32(b * cash_obs_scale), p * price_obs_scale, */
  float price_obs_scale;   /*                fl32(h) * hold_obs_scale (powers of two keep    */
  float hold_obs_scale;    /*                these exact)                                    */
} fm_env_config;

typedef struct fm_env fm_env;           /* opaque host handle */
typedef struct fm_ensemble fm_ensemble; /* opaque host handle */

/* Rollout options.  Trajectory pointers may each be NULL (not stored). */
typedef struct fm_rollout_opts {
  const float* d_actions;  /* [n_steps][N][D] float32: driven mode (the caller's actions are
                              executed); NULL: the ensemble acts on every state */
  float sigma;             /* Gaussian exploration noise added after averaging, >= 0 */
  uint64_t noise_key;      /* Philox4x64-10 key word; noise for env n, day t, stock d uses
                              counter (env_offset + n, t, d / 4, 0) */
  int64_t env_offset;      /* global index of env 0 (for sharding across devices) */
  int32_t path;            /* fm_path */
  float* d_obs_traj;       /* [n_steps][N][S] float32: state s_{t+1} after each step */
  float* d_act_traj;       /* [n_steps][N][D] float32: the action executed at each step */
  double* d_rew_traj;      /* [n_steps][N] float64 rewards */
  int32_t* d_qty_traj;     /* [n_steps][N][D] int32 executed shares (negative = sold) */
} fm_rollout_opts;

/* ---------------------------------------------------------------------------------------------
 * Environment (Section 4.2: a VecEnv of N SubEnvs, each with its own balance and holdings, on a
 * shared market path of prices and indicators).
 * ------------------------------------------------------------------------------------------- */

/* Device bytes the environment needs for its state (cash, total asset, cumulative reward as
 * float64 [N]; holdings int32 [D][N]; an action staging buffer float32 [N][D]).  Returns 0 for
 * an invalid configuration. */
size_t env_workspace_bytes(const fm_env_config* cfg);

/* Create an environment over the market arrays d_close [T+1][D] and d_ind [T+1][I][D]
 * (float32, indicator-major within a day).  d_workspace holds at least env_workspace_bytes(cfg)
 * bytes, 256-byte aligned.  The market arrays and the workspace must outlive the handle.
 * Nothing is enqueued: the state is undefined until env_reset or env_write_state. */
fm_status env_create(const fm_env_config* cfg, const float* d_close, const float* d_ind,
                     void* d_workspace, size_t workspace_bytes, hipStream_t stream, fm_env** out);

/* reset (Section 4.2): every sub-environment returns to day 0 with the initial cash and no
 * holdings.  Writes s_0 to d_obs [N][S] if it is not NULL. */
fm_status env_reset(fm_env* env, float* d_obs);

/* step and reward (Section 4.2) for one day: converts d_act [N][D] into integer orders
 * q = trunc(fl32(clamp(a, -1, 1) * hmax)) (NaN counts as 0), executes every sell (capped at the
 * holding) in ascending stock order and then every buy (the largest affordable k <= q) in
 * ascending stock order at the day-t close with proportional cost, advances to day t+1, and
 * writes r_t to d_reward [N], s_{t+1} to d_obs [N][S] and the executed shares to d_exec_qty
 * [N][D] (each optional except d_reward).  *h_done is set to 1 when day T is reached.
 * Returns FM_ERR_STATE if the environment is already at day T. */
fm_status env_step(fm_env* env, const float* d_act, float* d_obs, double* d_reward,
                   int32_t* d_exec_qty, int32_t* h_done);

/* A rollout of n_steps steps from the current day (Section 4.3: samples stored as T x N x D
 * tensors on the device).  ens may be NULL only in driven mode.  FM_PATH_FUSED needs a bfloat16
 * ensemble or driven mode.  Returns FM_ERR_STATE if the current day + n_steps exceeds T. */
fm_status env_rollout(fm_env* env, const fm_ensemble* ens, int32_t n_steps,
                      const fm_rollout_opts* opts);

/* Copy the state out to caller buffers (any may be NULL): cash, total asset v_t and cumulative
 * reward float64 [N], holdings int32 [N][D]; *h_day gets the current day. */
fm_status env_read_state(const fm_env* env, double* d_cash, int32_t* d_hold, double* d_asset,
                         double* d_cumrew, int32_t* h_day);

/* Overwrite the state (checkpoint resume).  All four buffers are required; 0 <= day <= T. */
fm_status env_write_state(fm_env* env, const double* d_cash, const int32_t* d_hold,
                          const double* d_asset, const double* d_cumrew, int32_t day);

/* The environment's current day (host-side bookkeeping; -1 for NULL). */
int32_t env_day(const fm_env* env);

/* Tuning (no effect on results): environments per workgroup of the environment kernels, 1..64;
 * 0 restores the size-based default.  A value whose LDS footprint does not fit is lowered at
 * launch.  Returns FM_ERR_INVALID for NULL or out-of-range values.  *h_tile (may be NULL) gets
 * the value in effect. */
fm_status env_set_tile(fm_env* env, int32_t envs_per_group, int32_t* h_tile);

/* Tuning (no effect on results): the environment-step kernel of env_step, driven rollouts and
 * the plain path's steps.  The row kernel (a 16-lane row per environment, one or two per wavefront) and
 * the lane kernel (one lane per environment, the whole trading chain in registers) take shapes
 * with n_stocks <= 32 and (2 + n_ind) * n_stocks < 256; the tile kernel takes every shape.
 * kernel 0 picks by shape and size: the row kernel up to n_envs = 12288 (for the plain path's
 * steps with at most 8 actors); above that the lane kernel for the plain path's steps, and for
 * env_step and driven rollouts the tile kernel up to 24575 environments and the lane kernel from
 * 24576; shapes outside the row and lane kernels' limits always take the tile kernel.  1 always
 * takes the tile kernel (env_set_tile's environments per workgroup); 2 the lane kernel and 3 the
 * row kernel whatever n_envs (3: the plain path's steps with more than 8 actors take the lane
 * kernel).  envs_per_wave: environments per wavefront of the lane kernel, 1..64 (0: by N, one
 * wavefront per SIMD), and of the row kernel, 1 or 2 (0 or above 2: 2; above 2 is refused with
 * kernel 3).  FM_ERR_INVALID for NULL or out-of-range values; FM_ERR_UNSUPPORTED for
 * kernel 2 or 3 on a shape it does not take.  Reset and observation always use the tile kernel. */
fm_status env_set_step_kernel(fm_env* env, int32_t kernel, int32_t envs_per_wave);

/* Tuning of the fused rollout (results stay within the bfloat16 tolerance; the environment
 * arithmetic is unchanged): schedule 0 picks, by shape and size, the resident schedule (weights
 * held on chip, eight environments per compute unit; K = 3, hidden 256, <= 31 stocks) when the
 * batch fits one workgroup per compute unit, else the streamed one (weights streamed from L2;
 * K = 3, hidden 256, <= 32 stocks), else the generic (runtime-shape) one; 1 skips the resident
 * schedule; 2 always takes the generic one; 3 takes the resident schedule whenever the shape
 * allows it, whatever N.  row_tiles 1 or 2 sets the streamed schedule's 16 or 32 MFMA rows per
 * workgroup (0: by N); tile_envs the environments per workgroup (resident <= 8, streamed <= 16 *
 * row_tiles; 0: fill the compute units).  FM_ERR_INVALID for NULL or out-of-range values. */
fm_status env_set_fused_tuning(fm_env* env, int32_t schedule, int32_t row_tiles, int32_t tile_envs);
void env_destroy(fm_env* env);

/* ---------------------------------------------------------------------------------------------
 * Ensemble (Section 5.2.1: the stock ensemble acts on the weighted average of its agents'
 * actions).  Each actor k is an MLP mu_k(s) = tanh(tanh(tanh(s W1 + b1) W2 + b2) W3 + b3) with
 * W1 [S][H], W2 [H][H], W3 [H][A]; the ensemble action is
 *   a = clip(sum_k w_k mu_k(s) + sigma * eps, -1, 1),
 * eps standard normal from Philox4x64-10 (Salmon et al., SC'11) and the Box-Muller transform.
 * ------------------------------------------------------------------------------------------- */

/* Device bytes for an ensemble that acts on at most max_batch states per call. */
size_t ensemble_workspace_bytes(int32_t n_actors, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                int32_t dtype, int32_t max_batch);

/* Pack the float32 master weights d_w (for k in 0..K-1: W1[S][H], b1[H], W2[H][H], b2[H],
 * W3[H][A], b3[A]) into d_workspace in the device layout of dtype (bfloat16 rounds the weight
 * matrices to nearest-even and keeps the biases float32).  h_mix [K] gives w_k (NULL: 1/K).
 * Limits: 1 <= K <= 8, 1 <= S <= 1024, H a multiple of 32 in 32..512, 1 <= A <= 128.  The
 * packing runs on stream and the call waits for it, so d_w may be released on return. */
fm_status ensemble_create(int32_t n_actors, int32_t in_dim, int32_t hidden, int32_t out_dim,
                          int32_t dtype, const float* d_w, const float* h_mix, int32_t max_batch,
                          void* d_workspace, size_t workspace_bytes, hipStream_t stream,
                          fm_ensemble** out);

/* Act on n states d_obs [n][S]: writes the ensemble mean to d_mean [n][A] (optional) and the
 * noisy, clipped action to d_act [n][A].  State row i is environment env_offset + i at day t for
 * the noise counter.  n <= max_batch.  Concurrent calls on one ensemble must use one stream. */
fm_status ensemble_act(const fm_ensemble* ens, const float* d_obs, int32_t n, float sigma,
                       uint64_t noise_key, int32_t t, int64_t env_offset, float* d_mean,
                       float* d_act, hipStream_t stream);

void ensemble_destroy(fm_ensemble* ens);

/* ---------------------------------------------------------------------------------------------
 * Evaluation (Section 6.1 metrics; Section 5.2.1 ensemble weights)
 * ------------------------------------------------------------------------------------------- */

/* Backtest metrics of every environment from its reward trajectory d_rew [n_steps][n_envs]
 * (float64, as env_rollout stores it).  The equity curve is v_0 = d_init_asset[n] (or init_asset
 * when d_init_asset is NULL), v_{t+1} = v_t + r_t / reward_scale, with period returns
 * rho_t = v_{t+1}/v_t - 1.  Writes d_out [n_envs][10] float64:
 *   0 cumulative return v_T/v_0 - 1        5 RoMaD = cumulative return / |max drawdown|
 *   1 annual return (v_T/v_0)^(P/T) - 1    6 Sortino = (mean rho - rf/P) / downside dev * sqrt(P)
 *   2 annual volatility sd(rho) * sqrt(P)  7 Calmar = annual return / |max drawdown|
 *   3 Sharpe (eq. 6) annualised by sqrt(P) 8 Omega = sum max(rho,0) / sum max(-rho,0)
 *   4 max drawdown min_t v_t/peak_t - 1    9 win/loss = #(rho>0) / #(rho<0)
 * sd is the sample (n-1) deviation, the downside deviation is sqrt(mean(min(rho - rf/P, 0)^2)),
 * P = periods_per_year, rf = risk_free (annual); a zero denominator gives inf or NaN. */
fm_status fm_backtest_metrics(const double* d_rew, int32_t n_steps, int32_t n_envs, double init_asset,
                              const double* d_init_asset, double reward_scale, double periods_per_year,
                              double risk_free, double* d_out, hipStream_t stream);

/* Ensemble weights from validation Sharpe ratios (Section 5.2.1): agents below min_sharpe get 0,
 * the others a softmax of their Sharpe ratios; if every agent is below, the best gets 1.
 * Host only; h_mix [n_actors] can be passed to ensemble_create. */
fm_status fm_sharpe_weights(const double* h_sharpe, int32_t n_actors, double min_sharpe, float* h_mix);

/* ---------------------------------------------------------------------------------------------
 * Uneven batch (Section 4.2: the vectorised environment is a set of independent sub-environments
 * with their own market and horizon; here G groups of them, each with its own stock count D_g,
 * environment count N_g, horizon and bfloat16 ensemble, run together).  One persistent kernel
 * launch per chunk of 64 days steps every group: workgroups take (group, tile) work items in
 * decreasing order of cost from a device counter until none is left.  The chunk launches can be
 * captured once in a hipGraph and replayed.
 * ------------------------------------------------------------------------------------------- */
typedef struct fm_batch fm_batch; /* opaque host handle */

typedef struct fm_batch_group {
  fm_env* env;               /* the group's environments (their stream is not used) */
  const fm_ensemble* ens;    /* bfloat16 ensemble with in_dim = the env's state width,
                                out_dim = its stock count, hidden <= 256 */
  int32_t n_steps;           /* days to advance, env day + n_steps <= T */
  float sigma;               /* exploration noise scale, finite, >= 0 */
  uint64_t noise_key;
  int64_t env_offset;        /* global index of the group's first environment (noise counter) */
  float* d_obs_traj;         /* optional [n_steps][N][S] */
  float* d_act_traj;         /* optional [n_steps][N][D] */
  double* d_rew_traj;        /* optional [n_steps][N] */
  int32_t* d_qty_traj;       /* optional [n_steps][N][D] */
} fm_batch_group;

/* Device workspace bytes for a batch of these groups (0 if the groups are invalid). */
size_t fm_batch_workspace_bytes(const fm_batch_group* h_groups, int32_t n_groups);

/* Validates the groups (1 <= n_groups <= 4096; every env and ensemble on the current device;
 * shapes as above), lays out the per-chunk group descriptors and work lists in d_workspace
 * (caller-owned, 256-byte aligned, >= fm_batch_workspace_bytes) and records each group's current
 * day: fm_batch_run requires the environments to be at those days again.  Synchronous. */
fm_status fm_batch_create(const fm_batch_group* h_groups, int32_t n_groups, void* d_workspace,
                          size_t workspace_bytes, hipStream_t stream, fm_batch** out);

/* Autotuner: times the first chunk under each candidate tile shape (16 or 32 environments per
 * work item; with 32, groups whose 32-row tile exceeds the LDS budget keep 16, in a launch of
 * their own) and persistent grid size, restores every group's state after each trial, and keeps
 * the fastest.  *h_rows and *h_blocks (may be NULL) get the choice.  Invalidates a captured
 * graph.  Trajectory buffers are overwritten by the trials. */
fm_status fm_batch_tune(fm_batch* batch, int32_t* h_rows, int32_t* h_blocks);

/* Sets the tile shape by hand instead of the autotuner: rows (16 or 32 environments per work item;
 * with 32, groups whose 32-row tile exceeds the LDS budget keep 16) and the persistent grid
 * (blocks, 1..65536 workgroups per launch).  Invalidates a captured graph. */
fm_status fm_batch_set_tiling(fm_batch* batch, int32_t rows, int32_t blocks);

/* Runs every group's n_steps on the batch's stream and advances each environment's day.
 * use_graph != 0 captures the chunk launches into a hipGraph on first use and replays it.
 * Returns FM_ERR_STATE if an environment is not at the day recorded by fm_batch_create. */
fm_status fm_batch_run(fm_batch* batch, int32_t use_graph);

void fm_batch_destroy(fm_batch* batch);

/* ---------------------------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------------------------- */

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* fm_last_error(void);

/* The Gaussian exploration noise exactly as the ensemble draws it: eps [n][D] float32 for
 * environments env_offset .. env_offset+n-1 at day t, and optionally the raw Philox4x64-10
 * blocks d_words [n][ceil(D/4)][4] (uint64).  Exposes the generator for checking. */
fm_status fm_noise(uint64_t noise_key, int64_t env_offset, int32_t n, int32_t t, int32_t n_stocks,
                   uint64_t* d_words, float* d_eps, hipStream_t stream);

/* Library version string. */
const char* fm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FINRL_MI_H */
