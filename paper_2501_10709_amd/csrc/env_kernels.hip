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

template <int DMAX>
struct TileCfg {
  static constexpr int kStride = DMAX + 4;                        // 16-byte rows for the chain
  static constexpr int kMaxM = DMAX <= 32 ? 64 : (2048 / DMAX);   // envs per workgroup
  static constexpr int kMaxI = 16;
  static constexpr int kMaxS = (kMaxI + 2) * DMAX + 1;
  static constexpr int kSlots = (kMaxS + kWave - 1) / kWave;      // state entries per lane
  static constexpr int kActRegs = kMaxM * DMAX / kWave;           // prefetched actions per lane
  static constexpr int kMktRegs = ((kMaxI + 2) * DMAX + kWave - 1) / kWave;
};

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

// Market entries of the step (it) in flat order: close[t] (D), close[t+1] (D), ind[t+1] (I*D).
__device__ __forceinline__ float market_entry(const EnvConst& C, int t, int tn, int i, bool with_trade) {
  const int D = C.D;
  if (i < D) return with_trade ? C.close[static_cast<size_t>(t) * D + i] : 0.0f;
  if (i < 2 * D) return C.close[static_cast<size_t>(tn) * D + (i - D)];
  return C.ind[static_cast<size_t>(tn) * C.I * D + (i - 2 * D)];
}

// Two wavefronts per workgroup.  Wavefront 0 fetches the next step's inputs into registers,
// runs the trading chains and moves the fetched inputs into LDS; wavefront 1 writes the step's
// results (states, quantities, rewards) from LDS to HBM.  Vector-memory completions are counted
// in issue order, so a wavefront that both stores and loads would wait for its stores every time
// it needs a loaded value; splitting the roles keeps the stores off the chain's critical path.
template <int DMAX, int MODE>
__global__ __launch_bounds__(2 * kWave) void env_tile_kernel(EnvConst C, EnvState st, StepArgs A) {
  using TC = TileCfg<DMAX>;
  constexpr int ST = TC::kStride;
  __shared__ __align__(16) float s_act[TC::kMaxM * ST];   // actions of the tile [m][d], zero-padded
  __shared__ float s_env[TC::kMaxM * ST];                 // per-env state entries [cash, h_0..]
  __shared__ int s_qty[TC::kMaxM * ST];
  __shared__ double s_rew[TC::kMaxM];
  __shared__ __align__(16) float s_px[DMAX];              // close of the trading day, zero-padded
  __shared__ __align__(16) float s_pn[DMAX];              // close of the new day, zero-padded
  __shared__ float s_mkt[2][(1 + TC::kMaxI) * DMAX];      // scaled new close + new indicators,
                                                          // double-buffered by step parity
  __shared__ float s_eps[TC::kMaxM * ST];

  const int lane = threadIdx.x & (kWave - 1);
  const bool loader = threadIdx.x < kWave;                // wavefront 0
  const int D = C.D, S = C.S, N = C.N;
  const int n0 = blockIdx.x * A.M;
  const int M = min(A.M, N - n0);
  const float inv_d = 1.0f / static_cast<float>(D);
  const int MD = M * D;
  const int n_mkt = (2 + C.I) * D;

  // Zero the padding once: columns >= D of the action rows and of the price rows.
  for (int i = threadIdx.x; i < TC::kMaxM * ST; i += 2 * kWave) s_act[i] = 0.0f;
  for (int i = threadIdx.x; i < DMAX; i += 2 * kWave) {
    s_px[i] = 0.0f;
    s_pn[i] = 0.0f;
  }

  // Store-wave plan for a state row: slot j covers entry f = lane + 64 j.
  // kind 0: shared market entry, 1: per-env entry s_env[idx], 2: none.
  int kind[TC::kSlots], eidx[TC::kSlots];
#pragma unroll
  for (int j = 0; j < TC::kSlots; ++j) {
    const int f = lane + kWave * j;
    kind[j] = 2;
    eidx[j] = 0;
    if (f < S) {
      if (f == 0) {
        kind[j] = 1;
      } else if (f <= D) {
        kind[j] = 0;
        eidx[j] = f - 1;
      } else if (f <= 2 * D) {
        kind[j] = 1;
        eidx[j] = f - D;
      } else {
        kind[j] = 0;
        eidx[j] = f - 1 - D;
      }
    }
  }

  // The tile's trading state, in the registers of wavefront 0's lanes 0..M-1.
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  int h[DMAX], x[DMAX];
  const bool active = loader && lane < M;
  const int n = n0 + lane;
#pragma unroll
  for (int d = 0; d < DMAX; ++d) {
    h[d] = 0;
    x[d] = 0;
  }
  if (MODE == kReset) {
    cash = C.init_cash;
  } else if (active) {
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
      if (d < D) h[d] = st.hold[static_cast<size_t>(d) * N + n];
  }

  const int n_iter = trades(MODE) ? A.n_steps : 1;
  // Inputs of step it are fetched into wavefront 0's registers one step ahead, then moved to LDS.
  float pa[TC::kActRegs], pm[TC::kMktRegs];
  auto fetch = [&](int it) {
    const int t = A.t0 + it;
    const int tn = trades(MODE) ? t + 1 : A.t0;
#pragma unroll
    for (int j = 0; j < TC::kMktRegs; ++j) {
      const int i = lane + kWave * j;
      pm[j] = i < n_mkt ? market_entry(C, t, tn, i, trades(MODE)) : 0.0f;
    }
    if (MODE == kGiven) {
      const float* src = A.act + (static_cast<size_t>(it) * N + n0) * D;
#pragma unroll
      for (int j = 0; j < TC::kActRegs; ++j) {
        const int i = lane + kWave * j;
        pa[j] = i < MD ? src[i] : 0.0f;
      }
    }
  };
  auto commit = [&](int it) {
    float* mkt = s_mkt[it & 1];
#pragma unroll
    for (int j = 0; j < TC::kMktRegs; ++j) {
      const int i = lane + kWave * j;
      if (i < D) {
        s_px[i] = pm[j];
      } else if (i < 2 * D) {
        s_pn[i - D] = pm[j];
        mkt[i - D] = pm[j] * C.price_scale;
      } else if (i < n_mkt) {
        mkt[i - D] = pm[j];
      }
    }
    if (MODE == kGiven) {
#pragma unroll
      for (int j = 0; j < TC::kActRegs; ++j) {
        const int i = lane + kWave * j;
        if (i < MD) {
          const int m = div_small(i, inv_d);
          s_act[m * ST + (i - m * D)] = pa[j];
        }
      }
    }
  };

  if (loader) {
    fetch(0);
    commit(0);
  }
  __syncthreads();

  for (int it = 0; it < n_iter; ++it) {
    const int t = A.t0 + it;
    if (loader) {
      if (it + 1 < n_iter) fetch(it + 1);

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
              if (4 * g + r < D) s_eps[m * ST + 4 * g + r] = z[r];
          }
        }
        for (int i = lane; i < MD; i += kWave) {
          const int m = div_small(i, inv_d);
          const int d = i - m * D;
          float acc = 0.0f;
          for (int k = 0; k < A.K; ++k)
            acc = acc + A.mix[k] * A.mu[(static_cast<size_t>(k) * N + n0) * D + i];
          float a = acc;
          if (A.sigma != 0.0f) a = acc + A.sigma * s_eps[m * ST + d];
          a = fminf(fmaxf(a, -1.0f), 1.0f);
          s_act[m * ST + d] = a;
        }
      }

      if (active) {
        if (trades(MODE)) {
          float a[DMAX], px[DMAX];
          lds_row<DMAX>(a, &s_act[lane * ST]);
          lds_row<DMAX>(px, s_px);
          trade<DMAX>(cash, h, x, a, px, C.hmax_f, C.one_m, C.one_p);
          float pn[DMAX];
          lds_row<DMAX>(pn, s_pn);
          const double v_new = portfolio_value<DMAX>(cash, h, pn);
          const double r = (v_new - asset) * C.reward_scale;
          cumrew = cumrew + r;
          asset = v_new;
          s_rew[lane] = r;
        } else if (MODE == kReset) {
          float pn[DMAX];
          lds_row<DMAX>(pn, s_pn);
          asset = portfolio_value<DMAX>(cash, h, pn);
        }
        s_env[lane * ST] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
          if (d < D) {
            s_env[lane * ST + 1 + d] = static_cast<float>(h[d]) * C.hold_scale;
            s_qty[lane * ST + d] = x[d];
          }
      }
    }
    __syncthreads();

    if (!loader) {
      // Results of step it.
      if (trades(MODE)) {
        if (A.rew && lane < M) A.rew[static_cast<size_t>(it) * N + n0 + lane] = s_rew[lane];
        if (MODE == kEnsemble && A.act_out) {  // single-step mode: s_act is not refilled
          float* dst = A.act_out + (static_cast<size_t>(it) * N + n0) * D;
          for (int i = lane; i < MD; i += kWave) {
            const int m = div_small(i, inv_d);
            dst[i] = s_act[m * ST + (i - m * D)];
          }
        }
        if (A.qty) {
          int* dst = A.qty + (static_cast<size_t>(it) * N + n0) * D;
          for (int i = lane; i < MD; i += kWave) {
            const int m = div_small(i, inv_d);
            dst[i] = s_qty[m * ST + (i - m * D)];
          }
        }
      }
      // States s_{t+1}: shared entries cached per slot, per-env entries from LDS.
      if (A.obs) {
        const float* mkt = s_mkt[it & 1];
        float* dst = A.obs + (static_cast<size_t>(it) * N + n0) * S;
        float mval[TC::kSlots];
#pragma unroll
        for (int j = 0; j < TC::kSlots; ++j) mval[j] = (kind[j] == 0) ? mkt[eidx[j]] : 0.0f;
        for (int m = 0; m < M; ++m) {
#pragma unroll
          for (int j = 0; j < TC::kSlots; ++j) {
            if (kind[j] != 2) {
              const float v = (kind[j] == 0) ? mval[j] : s_env[m * ST + eidx[j]];
              dst[static_cast<size_t>(m) * S + lane + kWave * j] = v;
            }
          }
        }
      }
    } else if (it + 1 < n_iter) {
      commit(it + 1);  // s_act, s_px, s_pn are free (the chain has read them); s_mkt is the other buffer
    }
    __syncthreads();
  }

  // Store the state back.
  if (MODE != kObserve && active) {
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
      if (d < D) st.hold[static_cast<size_t>(d) * N + n] = h[d];
  }
}

template <int DMAX, int MODE>
hipError_t launch_tile(const EnvConst& C, const EnvState& st, StepArgs A, hipStream_t stream) {
  A.M = min(A.M, TileCfg<DMAX>::kMaxM);
  const int grid = (C.N + A.M - 1) / A.M;
  hipLaunchKernelGGL((env_tile_kernel<DMAX, MODE>), dim3(grid), dim3(2 * kWave), 0, stream, C, st,
                     A);
  return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_tile(const EnvConst& C, const EnvState& st, const StepArgs& A,
                         hipStream_t stream) {
  if (C.D <= 8) return launch_tile<8, MODE>(C, st, A, stream);
  if (C.D <= 16) return launch_tile<16, MODE>(C, st, A, stream);
  if (C.D <= 32) return launch_tile<32, MODE>(C, st, A, stream);
  if (C.D <= 64) return launch_tile<64, MODE>(C, st, A, stream);
  if (C.D <= 128) return launch_tile<128, MODE>(C, st, A, stream);
  return hipErrorInvalidValue;
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
