// Environment kernels: reset, step (caller actions or ensemble means plus noise), the
// multi-step driven rollout, state copies, and the noise probe.
//
// Thread mapping.  A workgroup is one 64-lane wavefront that owns M consecutive environments
// (M <= 64).  Lane m < M runs environment n0+m's trading chain, which is serial in the stock
// index because cash after stock d decides the fill of stock d+1 (sells then buys, ascending).
// All 64 lanes stage the tile's actions from HBM into LDS and write the tile's states,
// executed quantities and actions back with consecutive lanes on consecutive addresses: a
// tile's rows are contiguous in the [N][.] layouts, so every wave-wide load or store covers a
// contiguous run of 256 bytes.  The state entries shared by all environments (prices and
// indicators of the new day) are read once per lane per step from LDS; only cash and holdings
// differ between the rows.
#include "device_common.h"
#include "launch.h"

namespace fm {

namespace {

constexpr int kWave = 64;
constexpr int kPrefetch = 8;  // registers per lane for the next step's inputs (512 values)

enum Mode { kReset = 0, kGiven = 1, kEnsemble = 2, kObserve = 3 };
constexpr bool trades(int mode) { return mode == kGiven || mode == kEnsemble; }

struct StepArgs {
  int t0;              // first day
  int n_steps;         // days to advance (kGiven may loop; kReset uses 0; kEnsemble uses 1)
  int M;               // envs per workgroup
  const float* act;    // kGiven: [n_steps][N][D]
  const float* mu;     // kEnsemble: [K][N][A] actor means, A == D
  const float* mix;    // kEnsemble: [K] weights w_k
  int K;
  float sigma;
  uint64_t noise_key;
  int64_t env_offset;
  float* obs;          // [n_steps][N][S] or [N][S] for reset, may be null
  float* act_out;      // [n_steps][N][D] or null
  double* rew;         // [n_steps][N] or null
  int* qty;            // [n_steps][N][D] or null
};

// Market entries of the step in flat order: close[t] (D), close[t+1] (D), ind[t+1] (I*D).
__device__ __forceinline__ float market_entry(const EnvConst& C, int t, int tn, int i, bool with_trade) {
  const int D = C.D;
  if (i < D) return with_trade ? C.close[static_cast<size_t>(t) * D + i] : 0.0f;
  if (i < 2 * D) return C.close[static_cast<size_t>(tn) * D + (i - D)];
  return C.ind[static_cast<size_t>(tn) * C.I * D + (i - 2 * D)];
}

// LDS bytes of one workgroup of env_tile_kernel.
__host__ __device__ inline size_t tile_lds_bytes(int M, int D, int I) {
  const size_t DS = D + 1;
  return sizeof(double) * M                // rewards
         + sizeof(double) * M * D * 3      // chain scratch: proceeds, debits, position values
         + sizeof(int) * M * D * 2         // chain scratch: whole orders, fills
         + sizeof(float) * M * DS * 2      // actions, two buffers
         + sizeof(float) * M * DS * 4      // hold, qty, env, eps
         + sizeof(float) * 4 * D           // closes of the trading day and the new day, two buffers
         + sizeof(float) * 2 * (1 + I) * D;  // new-day state entries, two buffers
}

// Three wavefronts per workgroup, one role each:
//   wavefront 0 (chain): the trading chains of the tile's M environments (lane m owns
//     environment m; holdings stay in LDS) -- LDS traffic only inside the step loop;
//   wavefront 1 (store): the step's results (states, quantities, rewards) from LDS to HBM;
//   wavefront 2 (fetch): the next step's inputs (actions, market rows) from HBM into the other
//     half of double-buffered LDS.
// Vector-memory completions are counted per wavefront in issue order, so a wavefront that mixed
// these roles would wait for stores and prefetches whenever it needed any loaded value; with the
// roles split, the chain never waits on HBM.  Loops over stocks stay rolled so that the whole
// step fits the instruction cache.
template <int MODE>
__global__ __launch_bounds__(3 * kWave) void env_tile_kernel(EnvConst C, EnvState st, StepArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1);
  const int role = threadIdx.x / kWave;  // 0 chain, 1 store, 2 fetch
  const int D = C.D, S = C.S, N = C.N, DS = D + 1;
  const int n0 = blockIdx.x * A.M;
  const int M = min(A.M, N - n0);
  const float inv_d = 1.0f / static_cast<float>(D);
  const int MD = M * D;
  const int n_mkt = (2 + C.I) * D;
  const int n_new = (1 + C.I) * D;  // scaled new close + new indicators

  double* s_rew = reinterpret_cast<double*>(smem);
  double* s_pro = s_rew + A.M;
  double* s_deb = s_pro + A.M * D;
  double* s_val = s_deb + A.M * D;
  int* s_qd = reinterpret_cast<int*>(s_val + A.M * D);
  int* s_kq = s_qd + A.M * D;
  float* s_act0 = reinterpret_cast<float*>(s_kq + A.M * D);  // two buffers of [M][DS]
  int* s_hold = reinterpret_cast<int*>(s_act0 + 2 * A.M * DS);
  int* s_qty = s_hold + A.M * DS;
  float* s_env = reinterpret_cast<float*>(s_qty + A.M * DS);  // [cash, h_0..h_{D-1}] per env
  float* s_eps = s_env + A.M * DS;
  float* s_px0 = s_eps + A.M * DS;   // two buffers of [D]
  float* s_pn0 = s_px0 + 2 * D;      // two buffers of [D]
  float* s_mkt0 = s_pn0 + 2 * D;     // two buffers of [n_new]

  // The tile's trading state: cash, asset, cumulative reward in the chain wavefront's registers,
  // holdings in LDS.
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  const bool active = role == 0 && lane < M;
  const int n = n0 + lane;
  int* hrow = s_hold + lane * DS;
  if (MODE == kReset) {
    cash = C.init_cash;
    if (active)
      for (int d = 0; d < D; ++d) hrow[d] = 0;
  } else if (active) {
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
    for (int d = 0; d < D; ++d) hrow[d] = st.hold[static_cast<size_t>(d) * N + n];
  }

  const int n_iter = trades(MODE) ? A.n_steps : 1;
  // Fetch wavefront: inputs of step it into buffer it & 1.  One flat index runs over the
  // trading-day closes (D), the new-day closes (D), the new-day indicators (I*D) and, in driven
  // mode, the tile's actions (M*D); each batch issues all its loads before any LDS write.
  auto fetch_into = [&](int it) {
    const int b = it & 1;
    const int t = A.t0 + it;
    const int tn = trades(MODE) ? t + 1 : A.t0;
    float* px = s_px0 + b * D;
    float* pn = s_pn0 + b * D;
    float* mkt = s_mkt0 + b * n_new;
    float* act = s_act0 + b * A.M * DS;
    const float* c_t = C.close + static_cast<size_t>(t) * D;
    const float* c_n = C.close + static_cast<size_t>(tn) * D;
    const float* ind = C.ind + static_cast<size_t>(tn) * C.I * D;
    // The tile's actions (driven mode); flat index i >= n_mkt is action i - n_mkt.
    const float* acts = (MODE == kGiven) ? A.act + (static_cast<size_t>(it) * N + n0) * D : C.close;

    const int total = n_mkt + ((MODE == kGiven) ? MD : 0);
    for (int i0 = 0; i0 < total; i0 += kPrefetch * kWave) {
      float v[kPrefetch];
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        const int i = i0 + lane + kWave * j;
        const float* src = i < D ? c_t + i : (i < 2 * D ? c_n + (i - D) : (i < n_mkt ? ind + (i - 2 * D) : acts + (i - n_mkt)));
        v[j] = (i < total && (i >= D || trades(MODE))) ? *src : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        const int i = i0 + lane + kWave * j;
        if (i >= total) {
        } else if (i < D) {
          px[i] = v[j];
        } else if (i < 2 * D) {
          pn[i - D] = v[j];
          mkt[i - D] = v[j] * C.price_scale;
        } else if (i < n_mkt) {
          mkt[i - D] = v[j];
        } else {
          const int k = i - n_mkt;
          const int m = div_small(k, inv_d);
          act[m * DS + (k - m * D)] = v[j];
        }
      }
    }
  };

  if (role == 2) fetch_into(0);
  __syncthreads();

  for (int it = 0; it < n_iter; ++it) {
    const int t = A.t0 + it;
    const int b = it & 1;
    float* s_act = s_act0 + b * A.M * DS;
    const float* s_px = s_px0 + b * D;
    const float* s_pn = s_pn0 + b * D;
    if (role == 0) {
      if (MODE == kEnsemble) {
        // Noise: one Philox block per (env, group of 4 stocks).
        const int G = (D + 3) >> 2;
        const float inv_g = 1.0f / static_cast<float>(G);
        if (A.sigma != 0.0f) {
          for (int i = lane; i < M * G; i += kWave) {
            const int m = div_small(i, inv_g);
            const int g = i - m * G;
            float z[4];
            noise_block(A.noise_key, static_cast<uint64_t>(A.env_offset + n0 + m),
                        static_cast<uint64_t>(t), static_cast<uint64_t>(g), z);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (4 * g + r < D) s_eps[m * DS + 4 * g + r] = z[r];
          }
        }
        wave_lds_sync();
        for (int i = lane; i < MD; i += kWave) {
          const int m = div_small(i, inv_d);
          const int d = i - m * D;
          float acc = 0.0f;
          for (int k = 0; k < A.K; ++k)
            acc = acc + A.mix[k] * A.mu[(static_cast<size_t>(k) * N + n0) * D + i];
          float a = acc;
          if (A.sigma != 0.0f) a = acc + A.sigma * s_eps[m * DS + d];
          a = fminf(fmaxf(a, -1.0f), 1.0f);
          s_act[m * DS + d] = a;
        }
      }
      // The chain: parallel pre-terms, serial cash recurrence per env, parallel post-terms.
      const ChainLds CL{s_act, s_hold, s_qty, s_env, s_px, s_pn, s_pro, s_deb, s_val, s_qd, s_kq};
      wave_lds_sync();
      if (trades(MODE)) {
        chain_pairs_a(CL, M, D, lane, kWave, inv_d, C.hmax_f, C.one_m, C.one_p);
        wave_lds_sync();
        if (active)
          chain_serial(cash, s_pro + lane * D, s_deb + lane * D, s_val + lane * D, s_qd + lane * D, s_px,
                       s_kq + lane * D, D, C.one_p);
        wave_lds_sync();
        chain_pairs_c(CL, M, D, lane, kWave, inv_d, C.hold_scale);
      } else {
        chain_pairs_hold(CL, M, D, lane, kWave, inv_d, C.hold_scale);
      }
      wave_lds_sync();
      if (active) {
        const double v_new = chain_value(cash, s_val + lane * D, D);
        if (trades(MODE)) {
          const double r = (v_new - asset) * C.reward_scale;
          cumrew = cumrew + r;
          s_rew[lane] = r;
        }
        if (MODE != kObserve) asset = v_new;
        s_env[lane * DS] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
      }
    } else if (role == 2 && it + 1 < n_iter) {
      fetch_into(it + 1);  // the other buffer: nobody reads it during this step
    }
    __syncthreads();

    if (role == 1) {
      // Results of step it: the tile's rows are contiguous in every [N][.] trajectory.
      const size_t row0 = static_cast<size_t>(it) * N + n0;
      if (trades(MODE)) {
        if (A.rew && lane < M) A.rew[row0 + lane] = s_rew[lane];
        if (MODE == kEnsemble && A.act_out)
          wave_store_row(A.act_out + row0 * D, MD, lane, [&](int i) {
            const int m = div_small(i, inv_d);
            return s_act[m * DS + (i - m * D)];
          });
        if (A.qty)
          wave_store_row(A.qty + row0 * D, MD, lane, [&](int i) {
            const int m = div_small(i, inv_d);
            return s_qty[m * DS + (i - m * D)];
          });
      }
      // States s_{t+1} = [cash, new closes, holdings, new indicators], one row per env.
      if (A.obs) {
        const float* mkt = s_mkt0 + b * n_new;
        const float inv_s = 1.0f / static_cast<float>(S);
        wave_store_row(A.obs + row0 * S, M * S, lane, [&](int e) {
          const int m = div_small(e, inv_s);
          const int f = e - m * S;
          const float* erow = s_env + m * DS;
          if (f == 0) return erow[0];
          if (f <= D) return mkt[f - 1];
          if (f <= 2 * D) return erow[f - D];
          return mkt[f - 1 - D];
        });
      }
    }
    __syncthreads();
  }

  // Store the state back.
  if (MODE != kObserve && active) {
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
    for (int d = 0; d < D; ++d) st.hold[static_cast<size_t>(d) * N + n] = hrow[d];
  }
}

template <int MODE>
hipError_t dispatch_tile(const EnvConst& C, const EnvState& st, StepArgs A, hipStream_t stream) {
  A.M = max(1, min(A.M, 64));
  const size_t lds = tile_lds_bytes(A.M, C.D, C.I);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(env_tile_kernel<MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  const int grid = (C.N + A.M - 1) / A.M;
  hipLaunchKernelGGL((env_tile_kernel<MODE>), dim3(grid), dim3(3 * kWave), lds, stream, C, st, A);
  return hipGetLastError();
}

__global__ void read_state_kernel(int N, int D, EnvState st, double* cash, int* hold,
                                  double* asset, double* cumrew) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  if (cash) cash[n] = st.cash[n];
  if (asset) asset[n] = st.asset[n];
  if (cumrew) cumrew[n] = st.cumrew[n];
  if (hold)
    for (int d = 0; d < D; ++d) hold[static_cast<size_t>(n) * D + d] = st.hold[static_cast<size_t>(d) * N + n];
}

__global__ void write_state_kernel(int N, int D, EnvState st, const double* cash, const int* hold,
                                   const double* asset, const double* cumrew) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  st.cash[n] = cash[n];
  st.asset[n] = asset[n];
  st.cumrew[n] = cumrew[n];
  for (int d = 0; d < D; ++d) st.hold[static_cast<size_t>(d) * N + n] = hold[static_cast<size_t>(n) * D + d];
}

__global__ void noise_kernel(uint64_t key, int64_t env_offset, int n, int t, int D,
                             uint64_t* words, float* eps) {
  const int G = (D + 3) >> 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * G) return;
  const int m = i / G, g = i - m * G;
  float z[4];
  uint64_t w[4];
  noise_block(key, static_cast<uint64_t>(env_offset + m), static_cast<uint64_t>(t),
              static_cast<uint64_t>(g), z, w);
  if (words)
    for (int r = 0; r < 4; ++r) words[static_cast<size_t>(i) * 4 + r] = w[r];
  for (int r = 0; r < 4; ++r)
    if (4 * g + r < D) eps[static_cast<size_t>(m) * D + 4 * g + r] = z[r];
}

}  // namespace

hipError_t launch_env_reset(const EnvConst& C, const EnvState& st, float* obs, int M,
                            hipStream_t stream) {
  StepArgs A{};
  A.t0 = 0;
  A.n_steps = 0;
  A.M = M;
  A.obs = obs;
  return dispatch_tile<kReset>(C, st, A, stream);
}

hipError_t launch_env_observe(const EnvConst& C, const EnvState& st, int day, float* obs, int M,
                              hipStream_t stream) {
  StepArgs A{};
  A.t0 = day;
  A.n_steps = 0;
  A.M = M;
  A.obs = obs;
  return dispatch_tile<kObserve>(C, st, A, stream);
}

hipError_t launch_env_given(const EnvConst& C, const EnvState& st, int t0, int n_steps,
                            const float* act, float* obs, double* rew, int* qty, int M,
                            hipStream_t stream) {
  StepArgs A{};
  A.t0 = t0;
  A.n_steps = n_steps;
  A.M = M;
  A.act = act;
  A.obs = obs;
  A.rew = rew;
  A.qty = qty;
  return dispatch_tile<kGiven>(C, st, A, stream);
}

hipError_t launch_env_ensemble_step(const EnvConst& C, const EnvState& st, int t,
                                    const float* mu, const float* mix, int K, float sigma,
                                    uint64_t key, int64_t env_offset, float* obs, float* act_out,
                                    double* rew, int* qty, int M, hipStream_t stream) {
  StepArgs A{};
  A.t0 = t;
  A.n_steps = 1;
  A.M = M;
  A.mu = mu;
  A.mix = mix;
  A.K = K;
  A.sigma = sigma;
  A.noise_key = key;
  A.env_offset = env_offset;
  A.obs = obs;
  A.act_out = act_out;
  A.rew = rew;
  A.qty = qty;
  return dispatch_tile<kEnsemble>(C, st, A, stream);
}

hipError_t launch_read_state(const EnvConst& C, const EnvState& st, double* cash, int* hold,
                             double* asset, double* cumrew, hipStream_t stream) {
  hipLaunchKernelGGL(read_state_kernel, dim3((C.N + 255) / 256), dim3(256), 0, stream, C.N, C.D,
                     st, cash, hold, asset, cumrew);
  return hipGetLastError();
}

hipError_t launch_write_state(const EnvConst& C, const EnvState& st, const double* cash,
                              const int* hold, const double* asset, const double* cumrew,
                              hipStream_t stream) {
  hipLaunchKernelGGL(write_state_kernel, dim3((C.N + 255) / 256), dim3(256), 0, stream, C.N, C.D,
                     st, cash, hold, asset, cumrew);
  return hipGetLastError();
}

hipError_t launch_noise(uint64_t key, int64_t env_offset, int n, int t, int D, uint64_t* words,
                        float* eps, hipStream_t stream) {
  const int total = n * ((D + 3) >> 2);
  hipLaunchKernelGGL(noise_kernel, dim3((total + 255) / 256), dim3(256), 0, stream, key,
                     env_offset, n, t, D, words, eps);
  return hipGetLastError();
}

}  // namespace fm
