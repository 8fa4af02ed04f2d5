/*
 * learner.h -- C ABI of the learner that consumes the rollout's samples on the GPU.
 *
 * The training loop of Section 3.2 alternates a simulation phase (the rollout, finrl_mi.h) with
 * a learning phase; Section 4.1 estimates the policy gradient from the sampled trajectories by
 * the Monte-Carlo sum of eq. (4):
 *     grad J(theta_i) = (1/N) sum_n sum_t R(tau_n) grad log pi_i(a_t^n | s_t^n),
 * and Section 5.1 adds an agent-diversity term to agent i's objective, eq. (5): the loss becomes
 * L - lambda sum_{j != i} KL(pi_j || pi_i).  fm_policy_gradient returns the gradient of
 *     J_i = (1/N) sum_{n,t} R_n log pi_i(a|s) + lambda/(N T) sum_{t,n} sum_{j != i} KL(pi_j || pi_i)
 * with respect to agent i's parameters, where pi_k(a|s) = N(mu_k(s), sigma^2 I), mu_k the actor
 * network (tanh after every layer), R_n = sum_t r_t^n (rewards as stored, summed in t order), and
 * a = abar(s) + sigma eps the action the rollout sampled before clipping: abar = sum_k w_k mu_k(s)
 * and eps regenerated from the rollout's noise generator (key, env_offset + n, day t0 + t).  For equal
 * sigma, KL(pi_j || pi_i) = |mu_j - mu_i|^2 / (2 sigma^2).  Arithmetic is float32 with
 * fixed summation orders (the result is reproducible bit for bit; tanh is evaluated from one
 * exponential and one reciprocal, absolute error below 1e-6); the per-row terms are summed over
 * rows in float64 before the result is rounded to float32.
 *
 * Conventions follow finrl_mi.h (caller-owned d_* buffers, no device allocation, validation
 * before anything is enqueued, FM_ERR_* statuses with fm_last_error()).
 */
#ifndef LEARNER_H
#define LEARNER_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "finrl_mi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Device workspace bytes for K actors S -> H -> H -> A and T x N samples (0 if invalid:
 * 1 <= K <= 8, 1 <= S, H <= 1024, 1 <= A <= 128, N, T >= 1, N*T <= 2^26). */
size_t fm_pg_workspace_bytes(int32_t K, int32_t S, int32_t H, int32_t A, int32_t N, int32_t T);

/* d_w: float32 master weights of all K actors, per actor W1[S][H], b1[H], W2[H][H], b2[H],
 * W3[H][A], b3[A] (x W convention).  h_mix: host [K] ensemble weights w_k (NULL = 1/K).
 * agent: i in 0..K-1.  d_states: [T][N][S] float32, the state each action was taken in (s_0 from
 * reset, then the stored next states).  d_rew: [T][N] float64 rewards.  sigma > 0 and noise_key,
 * env_offset: those of the rollout.  t0 >= 0: the day of the first sample row (its state s_0 is the
 * state on day t0; 0 for a rollout from reset, the day read by env_day for one resumed with
 * env_write_state or run in pieces); row t's noise is the one drawn on day t0 + t.  lambda_kl >= 0.
 * d_grad: float32, one actor's parameters in the layout of d_w (overwritten).
 * abar is recomputed from the float32 master weights: for a rollout whose ensemble ran in
 * bfloat16 the reconstructed sample differs from the one drawn by the bfloat16 arithmetic error of
 * abar (about 3e-3 at 211-256-256-30), i.e. the gradient is taken at the float32 policy's samples.
 * Enqueued on stream; returns without synchronising. */
fm_status fm_policy_gradient(int32_t K, int32_t S, int32_t H, int32_t A, const float* d_w, const float* h_mix,
                             int32_t agent, const float* d_states, const double* d_rew, int32_t N, int32_t T,
                             float sigma, uint64_t noise_key, int64_t env_offset, int32_t t0, float lambda_kl,
                             float* d_grad, void* d_workspace, size_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under stream or graph capture, serving
 * loops that must not allocate, harnesses that forbid it): fm_policy_gradient with its workspace
 * in device memory the library holds -- one array of FM_PG_NOALLOC_MAX_BYTES per device, kept
 * until the process ends -- instead of d_workspace.  Same arguments, results and errors as
 * fm_policy_gradient; FM_ERR_INVALID if fm_pg_workspace_bytes(K, S, H, A, N, T) exceeds
 * FM_PG_NOALLOC_MAX_BYTES (about 13,000 sample rows at 211-256-256-30, K = 3).  Allocates nothing
 * (no device or pinned memory, no library allocator).  Every call on a device uses that device's
 * one array: calls that overlap on one device (other streams, other host threads) race and must be
 * serialised by the caller. */
#define FM_PG_NOALLOC_MAX_BYTES ((size_t)32 << 20)
fm_status fm_policy_gradient_noalloc(int32_t K, int32_t S, int32_t H, int32_t A, const float* d_w,
                                     const float* h_mix, int32_t agent, const float* d_states, const double* d_rew,
                                     int32_t N, int32_t T, float sigma, uint64_t noise_key, int64_t env_offset,
                                     int32_t t0, float lambda_kl, float* d_grad, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LEARNER_H */
