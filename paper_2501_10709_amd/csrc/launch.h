// Host-side launchers of the library's kernels (internal; the public ABI is finrl_mi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.h"
#include "mlp_device.h"

namespace fm {

// Environment kernels (env_kernels.hip).  M = environments per 64-lane workgroup.
hipError_t launch_env_reset(const EnvConst& C, const EnvState& st, float* obs, int M,
                            hipStream_t stream);
hipError_t launch_env_observe(const EnvConst& C, const EnvState& st, int day, float* obs, int M,
                              hipStream_t stream);
hipError_t launch_env_given(const EnvConst& C, const EnvState& st, int t0, int n_steps,
                            const float* act, float* obs, double* rew, int* qty, int M,
                            hipStream_t stream);
hipError_t launch_env_ensemble_step(const EnvConst& C, const EnvState& st, int t,
                                    const float* mu, const float* mix, int K, float sigma,
                                    uint64_t key, int64_t env_offset, float* obs, float* act_out,
                                    double* rew, int* qty, int M, hipStream_t stream);
// One lane per environment (env_lane.hip): the trading chain in registers, for D <= 32 and
// (2 + I) * D < 256.  envs_per_wave 0: by N (one wavefront per SIMD, up to 64 environments).
bool env_lane_shape(const EnvConst& C);
hipError_t launch_env_lane_given(const EnvConst& C, const EnvState& st, int t0, int n_steps, const float* act,
                                 float* obs, double* rew, int* qty, int envs_per_wave, hipStream_t stream);
hipError_t launch_env_lane_ensemble_step(const EnvConst& C, const EnvState& st, int t, const float* mu,
                                         const float* mix, int K, float sigma, uint64_t key, int64_t env_offset,
                                         float* obs, float* act_out, double* rew, int* qty, int envs_per_wave,
                                         hipStream_t stream);
// Row variant (env_lane.hip): one or two environments per wavefront (envs_per_wave; 0: by N),
// a 16-lane row each; same shapes.
hipError_t launch_env_row_given(const EnvConst& C, const EnvState& st, int t0, int n_steps, const float* act,
                                float* obs, double* rew, int* qty, int envs_per_wave, hipStream_t stream);
hipError_t launch_env_row_ensemble_step(const EnvConst& C, const EnvState& st, int t, const float* mu,
                                        const float* mix, int K, float sigma, uint64_t key, int64_t env_offset,
                                        float* obs, float* act_out, double* rew, int* qty, int envs_per_wave,
                                        hipStream_t stream);
hipError_t launch_read_state(const EnvConst& C, const EnvState& st, double* cash, int* hold,
                             double* asset, double* cumrew, hipStream_t stream);
hipError_t launch_write_state(const EnvConst& C, const EnvState& st, const double* cash,
                              const int* hold, const double* asset, const double* cumrew,
                              hipStream_t stream);
hipError_t launch_noise(uint64_t key, int64_t env_offset, int n, int t, int D, uint64_t* words,
                        float* eps, hipStream_t stream);

// Ensemble kernels (ensemble_kernels.hip).
hipError_t launch_pack_matrix(int dtype, const float* w, int kin, int nout, int kin_pad,
                              int nout_pad, void* out, hipStream_t stream);
hipError_t launch_copy_pad(const float* src, int n, int n_pad, float* dst, hipStream_t stream);
// Split first layer: the per-environment rows of W1 [S][H] (row 0, rows A+1..2A) as bfloat16
// MFMA fragments over ke_pad rows; the market rows (1..A, 2A+1..S-1) as bfloat16 [S-1-A][H].
hipError_t launch_pack_env_rows(const float* w1, int A, int H, int ke_pad, void* out, hipStream_t stream);
hipError_t launch_gather_market_rows(const float* w1, int S, int H, int A, __bf16* out, hipStream_t stream);
hipError_t launch_mlp(int dtype, const EnsDev& E, const float* obs, int n, float* mu,
                      hipStream_t stream);
hipError_t launch_combine(int K, int n, int A, const float* mu, const float* mix, float sigma,
                          uint64_t key, int t, int64_t env_offset, float* mean, float* act,
                          hipStream_t stream);

// Backtest metrics (metrics_kernels.hip).
hipError_t launch_metrics(const double* rew, int T, int N, double v0, const double* v0s,
                          double reward_scale, double periods_per_year, double risk_free,
                          double* out, hipStream_t stream);

}  // namespace fm
