// The fused rollout: ensemble MLP (bfloat16 MFMA), noise, trading, reward and next state for
// every step of a rollout in one launch (fused_rollout.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "device_common.h"
#include "mlp_device.h"

namespace fm {

// Steps per launch of the streamed schedule; its per-chunk scratch holds this many days.
constexpr int kFusedChunk = 64;
// Scratch floats of the streamed schedule for N environments and D stocks: the chunk's noise
// [kFusedChunk][N][D] and market table [kFusedChunk][8][512] (any supported K, H).
inline size_t fused_eps_floats(size_t N, size_t D) { return static_cast<size_t>(kFusedChunk) * N * D; }
inline size_t fused_table_floats() { return static_cast<size_t>(kFusedChunk) * 8 * 512; }

// Arguments of a fused launch over a chunk of steps.
struct FusedArgs {
  int t0, n_steps;
  float sigma;
  uint64_t key;
  int64_t env_offset;
  float* obs_traj;
  float* act_traj;
  double* rew_traj;
  int* qty_traj;
  const float* eps;  // streamed and resident schedules: the chunk's noise [n_steps][N][D]
  const float* mt;   // streamed and resident schedules: the chunk's layer-1 market shares [n_steps][K][H]
  int tile_envs = 0; // streamed and resident schedules: environments per workgroup
};

// Environments per workgroup of the resident schedule (one compute unit each).
constexpr int kResRows = 8;

// Rows (environments) per workgroup of the fused kernel: 16 * row_tiles.
struct FusedTuning {
  int row_tiles = 0;  // streamed: 0 chooses from the problem size
  int schedule = 0;   // 0: resident when the shape allows and N fills at most one workgroup per
                      // compute unit, else streamed when the shape allows; 1: streamed when the
                      // shape allows; 2: always the generic schedule; 3: resident whenever the
                      // shape allows
  int tile_envs = 0;  // resident / streamed: environments per workgroup, 0: fill the compute units
};

// True when the streamed MLP schedule handles this ensemble and environment.
bool fused_streamed_shape(const EnvConst& C, const EnsDev& E);
// True when the resident schedule (weights held on chip) handles them.
bool fused_resident_shape(const EnvConst& C, const EnsDev& E);

// The per-chunk inputs of the streamed and resident schedules, for days t .. t+n-1: the market
// table mt[c][k][j] (actor k's layer-1 share of day t+c's market entries, bias included) and,
// when sigma != 0, the noise eps[c][n][d].
hipError_t launch_chunk_inputs(const EnvConst& C, const EnsDev& E, int t, int n, float sigma, uint64_t key,
                               int64_t env_offset, float* eps_chunk, float* mt_chunk, hipStream_t stream);
// The resident schedule over F's steps, chunk by chunk (fused_resident.hip).
hipError_t launch_resident(const EnvConst& C, const EnvState& st, const EnsDev& E, FusedArgs F, float* eps_chunk,
                           float* mt_chunk, hipStream_t stream);

// Returns hipSuccess and leaves *why empty on success; sets *why for unsupported shapes.
hipError_t launch_fused_rollout(const EnvConst& C, const EnvState& st, const EnsDev& E, int t0,
                                int n_steps, float sigma, uint64_t key, int64_t env_offset,
                                float* obs_traj, float* act_traj, double* rew_traj, int* qty_traj,
                                float* eps_chunk, float* mt_chunk, hipStream_t stream, std::string* why,
                                FusedTuning tune = FusedTuning());

// Batched persistent rollout of uneven groups (generic schedule, hidden size 256, K <= 8; the
// first layer split into per-environment rows and a per-day market table when the ensemble
// packs it so).
// rows: environments per work item (16 or 32).  A group descriptor is an opaque block of
// batched_group_desc_bytes() bytes, filled on the host and copied to the device.
size_t batched_lds_bytes(int rows, const EnvConst& C, const EnsDev& E);
size_t batched_group_desc_bytes();
// mt: the group's market-table slot ([kFusedChunk][K][H] floats, refilled before each chunk by
// launch_market_table) when the ensemble splits its first layer, else ignored.
void batched_group_desc(const EnvConst& C, const EnvState& st, const EnsDev& E, int t0, int n_steps, float sigma,
                        uint64_t key, int64_t env_offset, float* obs_traj, float* act_traj, double* rew_traj,
                        int* qty_traj, const float* mt, void* out);
// The market table mt[c][k][j] of days t .. t+n-1 (actor k's layer-1 share of day t+c's market
// entries, bias included), for ensembles that split their first layer.
hipError_t launch_market_table(const EnvConst& C, const EnsDev& E, int t, int n, float* mt, hipStream_t stream);
// The batched kernels' dynamic LDS limit: raised to lds (<= batched_max_lds()) outside any
// stream capture.
size_t batched_max_lds();
hipError_t prepare_batched(size_t lds);
// items: int2 (group, tile) pairs; counter: one int of device scratch.
hipError_t launch_batched(int rows, int blocks, size_t lds, const void* groups, const int* items, int n_items,
                          int* counter, hipStream_t stream);

}  // namespace fm
