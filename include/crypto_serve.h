/*
 * crypto_serve.h -- C ABI of the single-asset crypto task served with continuous batching.
 *
 * The crypto task of the paper (Sections 3.1 and 5.2.2) trades one asset with discrete actions
 * chosen by an ensemble of value-based agents.  Here each environment holds one asset position
 * h in {-1, 0, +1} units and float64 cash b; action j in {0, 1, 2} moves the position to
 * h' = j - 1 at the tick's mid price p, paying (|h' - h| p) fee; the reward is
 * v_{t+1} - v_t with v = b + h p (Section 3.1, Reward).  The agents' input is the state
 * [b 2^-17, p 2^-16, h, f] (Section 3.1, State) with 13 market features f per tick, and each
 * agent is a ReLU network 16 -> 128 -> 128 -> 3 whose outputs are the three actions' values.
 * The ensemble either averages the agents' softmax probabilities (weights w_k) and takes the
 * argmax, or takes the majority vote of the agents' own argmax actions (Section 5.2.2); ties go
 * to the lowest action.  With probability eps an environment explores: Philox4x64-10 with key
 * (request key, 1) and counter (n, t, 0, 0) gives u = ((w0 >> 41) + 0.5) 2^-23; it explores iff
 * u < eps and then takes action (w1 >> 32) mod 3.
 *
 * Serving: requests (a number of environments, a horizon in ticks, a start tick and stride into
 * a shared tick table, an exploration key) are queued by fm_serve_submit and run by repeated
 * fm_serve_step calls.  Each step admits queued requests in arrival order while the caller's
 * device pool has room for their state (fm_serve_request_bytes) and the active-environment and
 * active-request limits allow, then launches one chunk of chunk_ticks ticks for every active
 * request in a single persistent kernel, whose workgroups take (request, tile) items from a
 * device counter.  A request finishes inside the chunk that reaches its horizon; its pool space
 * is reused from the next chunk on (the stream orders the two).  Results are per-environment
 * running backtest statistics (Section 6.1 metrics are formed from them on the host).
 *
 * Conventions follow finrl_mi.h: d_* device buffers and h_* host memory are owned by the caller,
 * the library allocates no device memory (it allocates pinned host staging for the per-chunk
 * work lists at create), arguments are validated before anything is enqueued, and failures
 * return a status with the message in fm_last_error().  Calls on one server must not overlap.
 */
#ifndef CRYPTO_SERVE_H
#define CRYPTO_SERVE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "finrl_mi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fm_ensemble_rule {
  FM_RULE_AVG_SOFTMAX = 0,   /* argmax of sum_k w_k softmax(Q_k) */
  FM_RULE_MAJORITY_VOTE = 1  /* most frequent argmax_j Q_k[j] over the agents */
} fm_ensemble_rule;

/* Per-environment state and result (64 bytes).  value = b + h p at the current tick; peak and
 * max_drawdown track v over the ticks run (max_drawdown = largest peak - v, in cash units);
 * trades counts ticks on which the position changed; ticks = ticks run. */
typedef struct fm_crypto_result {
  double cash, value, sum_r, sum_r2, peak, max_drawdown;
  int32_t position, trades;
  int64_t ticks;
} fm_crypto_result;

typedef struct fm_serve fm_serve; /* opaque host handle */

typedef struct fm_serve_config {
  int32_t device;
  /* Tick table, read-only while the server lives. */
  const double* d_mid;         /* [n_ticks] mid prices, > 0 */
  const float* d_feat;         /* [n_ticks][16] features in columns 3..15 (0..2 ignored) */
  int64_t n_ticks;             /* >= 2 */
  /* Agents. */
  int32_t n_agents;            /* K: 1, 3 or 5 */
  const float* h_weights;      /* float32, per agent: W1[16][128], b1[128], W2[128][128], b2[128],
                                  W3[128][3], b3[3] (x W convention); W1..W3 are rounded to
                                  bfloat16 (nearest, ties to even), biases stay float32 */
  const float* h_mix;          /* [K] softmax-average weights, NULL = 1/K each */
  int32_t rule;                /* fm_ensemble_rule */
  float eps;                   /* exploration probability in [0, 1] */
  double fee;                  /* proportional fee, [0, 1) */
  double cash0;                /* initial cash, finite */
  /* Scheduling. */
  int32_t tile_rows;           /* environments per work item: 16 or 64 */
  int32_t chunk_ticks;         /* ticks per launch, 1..65536 */
  int32_t max_requests;        /* active requests, 1..65536 */
  int64_t max_active_envs;     /* active environments, >= 1 */
  int32_t grid;                /* persistent workgroups per launch, 0 = one per compute unit */
  void* d_pool;                /* per-environment state of active requests (256-byte aligned) */
  size_t pool_bytes;
  void* d_workspace;           /* packed agents and work lists, >= fm_serve_workspace_bytes */
  size_t workspace_bytes;
} fm_serve_config;

typedef struct fm_serve_request {
  int32_t n_envs;              /* 1..2^24 */
  int32_t stride;              /* environment n starts at start_tick + n * stride, >= 0 */
  int64_t horizon;             /* ticks per environment, >= 1 */
  int64_t start_tick;          /* start_tick + (n_envs-1) stride + horizon <= n_ticks - 1 */
  uint64_t key;                /* exploration stream */
  fm_crypto_result* d_result;  /* [n_envs], written by the chunk that reaches the horizon */
  int8_t* d_act;               /* optional [horizon][n_envs] chosen actions 0..2 */
  float* d_prob;               /* optional [horizon][n_envs][3]: the averaged probabilities, or
                                  vote counts / K under the majority vote */
} fm_serve_request;

/* Pool bytes a request of n_envs environments occupies while active (0 if n_envs < 1). */
size_t fm_serve_request_bytes(int32_t n_envs);

/* Device workspace bytes for this configuration (0 if it is invalid). */
size_t fm_serve_workspace_bytes(const fm_serve_config* cfg);

/* Validates the configuration, packs the agents into d_workspace (bfloat16 MFMA fragments) on
 * `stream` and synchronises it.  The market, pool and workspace must stay alive until destroy. */
fm_status fm_serve_create(const fm_serve_config* cfg, hipStream_t stream, fm_serve** out);

/* Queues a request (validated here; FM_ERR_INVALID if it can never fit the pool or the limits).
 * *id gets its identifier (0, 1, 2, ... in submission order).  Host only. */
fm_status fm_serve_submit(fm_serve* s, const fm_serve_request* req, int64_t* id);

/* One scheduling step: admit what fits, launch one chunk for every active request on `stream`
 * (always the same stream for a server), retire the requests that finish in it.  At most two
 * chunks are in flight: the call waits for the chunk before the previous one.  *n_active and
 * *n_queued (may be NULL) get the counts after the step; nothing is launched if no request is
 * active. */
fm_status fm_serve_step(fm_serve* s, hipStream_t stream, int32_t* n_active, int32_t* n_queued);

/* Identifiers of requests whose results are complete in device memory, in completion order, up
 * to cap of them; *n gets how many were written.  wait != 0 blocks until every launched chunk
 * has completed first. */
fm_status fm_serve_poll(fm_serve* s, int32_t wait, int64_t* h_ids, int32_t cap, int32_t* n);

/* Waits for launched work and frees the host resources. */
void fm_serve_destroy(fm_serve* s);

#ifdef __cplusplus
}
#endif

#endif /* CRYPTO_SERVE_H */
