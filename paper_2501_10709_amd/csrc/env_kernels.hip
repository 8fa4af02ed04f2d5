// Environment kernels: reset, step (caller actions or ensemble means plus noise), the
// multi-step driven rollout, state copies, and the noise probe.
//
// Thread mapping.  A workgroup owns M consecutive environments (M <= 64) and runs three
// wavefronts with one role each (below).  Lane m < M of the chain wavefront runs environment
// n0+m's trading chain, which is serial in the stock index because cash after stock d decides
// the fill of stock d+1 (sells then buys, ascending); the cash-independent terms are computed by
// all 64 lanes over the (env, stock) pairs.  A tile's rows are contiguous in every [N][.] layout,
// so the loads of its actions and the stores of its states, quantities and actions are
// wave-wide runs of consecutive addresses.
#include "device_common.h"
#include "launch.h"

namespace fm {

namespace {

constexpr int kWave = 64;
constexpr int kStage = 16;       // registers per fetch lane holding a later step's inputs
constexpr int kInBufs = 3;       // input buffers: fetched (t+1), in use (t), being stored (t-1)
constexpr size_t kMaxLds = 160 * 1024;

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

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// One step's inputs as one LDS buffer, in the order of the flat fetch index:
// [close[t] (D) | close[t+1] (D) | ind[t+1] (I*D) | the tile's actions (M*D)], at least DP floats.
__host__ __device__ inline size_t in_buf_floats(int M, int D, int I) {
  const size_t n = static_cast<size_t>(2 + I) * D + static_cast<size_t>(M) * D;
  const size_t dp = ChainShape::of(D).DP;
  return align16(sizeof(float) * (n > dp ? n : dp)) / sizeof(float);
}

// LDS bytes of one workgroup of env_tile_kernel.
__host__ __device__ inline size_t tile_lds_bytes(int M, int D, int I) {
  const ChainShape Z = ChainShape::of(D);
  return Z.scratch_bytes(M)                                   // chain scratch
         + 2 * align16(sizeof(double) * M)                    // rewards, two buffers
         + align16(sizeof(int) * M * D)                       // holdings
         + align16(sizeof(float) * M * D)                     // noise
         + 2 * align16(sizeof(int) * M * D)                   // executed shares, two buffers
         + 2 * align16(sizeof(float) * M * Z.DS)              // state entries, two buffers
         + kInBufs * sizeof(float) * in_buf_floats(M, D, I);  // inputs
}

// Three wavefronts per workgroup, one role each:
//   wavefront 0 (chain): step t of the tile's M environments (holdings stay in LDS);
//   wavefront 1 (store): the results of step t-1 (states, quantities, rewards) from LDS to HBM;
//   wavefront 2 (fetch): writes step t+1's inputs into LDS from registers and requests step
//     t+2's inputs from HBM into those registers.
// One workgroup barrier per step separates them: the results are double-buffered and the inputs
// triple-buffered, so no role waits for another inside a step.  Vector-memory completions are
// counted per wavefront in issue order, so with the roles split the chain never waits on HBM and
// the store wavefront never waits for the fetches.
//
// OCC is the number of workgroups a compute unit is meant to hold: 1 (latency: all registers,
// cash chunks of 8 stocks) when the grid does not fill the GPU; 2 or 3 (throughput: at most 256
// or 168 registers per lane, chunks of 4, and for 3 half the fetch staging registers) when
// there are more tiles than compute units and that many workgroups fit the LDS.
template <int MODE, int OCC>
__global__ __launch_bounds__(3 * kWave, OCC) void env_tile_kernel(EnvConst C, EnvState st, StepArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1);
  const int role = threadIdx.x / kWave;  // 0 chain, 1 store, 2 fetch
  const int D = C.D, S = C.S, N = C.N, DS = D + 1;
  const ChainShape Z = ChainShape::of(D);
  const int MM = A.M;                    // rows allocated per workgroup
  const int n0 = blockIdx.x * MM;
  const int M = min(MM, N - n0);         // rows of this workgroup
  const int MD = M * D;
  const int n_mkt = (2 + C.I) * D;
  const int IB = static_cast<int>(in_buf_floats(MM, D, C.I));

  ChainLds CL{};
  unsigned char* p = CL.carve_scratch(smem, Z, MM);
  double* s_rew0 = reinterpret_cast<double*>(p);
  const int RB = static_cast<int>(align16(sizeof(double) * MM) / sizeof(double));
  p += 2 * align16(sizeof(double) * MM);
  int* s_hold = reinterpret_cast<int*>(p);
  p += align16(sizeof(int) * MM * D);
  float* s_eps = reinterpret_cast<float*>(p);
  p += align16(sizeof(float) * MM * D);
  int* s_qty0 = reinterpret_cast<int*>(p);
  const int QB = static_cast<int>(align16(sizeof(int) * MM * D) / sizeof(int));
  p += 2 * align16(sizeof(int) * MM * D);
  float* s_env0 = reinterpret_cast<float*>(p);
  const int EB = static_cast<int>(align16(sizeof(float) * MM * DS) / sizeof(float));
  p += 2 * align16(sizeof(float) * MM * DS);
  float* s_in0 = reinterpret_cast<float*>(p);

  // The tile's trading state: cash, asset, cumulative reward in the chain wavefront's registers,
  // holdings in LDS.
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  const bool active = role == 0 && lane < M;
  const int n = n0 + lane;
  int* hrow = s_hold + lane * D;
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
  const int total = n_mkt + ((MODE == kGiven) ? MD : 0);  // fetched floats per step
  const int staged = min(total, (OCC >= 4 ? kStage / 4 : OCC >= 3 ? kStage / 2 : kStage) * kWave);

  // Fetch wavefront.  Flat index i of step it's inputs: close[t] (D; zeros when not trading),
  // close[tn] (D), ind[tn] (I*D), then, driven, the tile's actions (M*D) -- which is also the
  // layout of the LDS buffer.
  auto src_of = [&](int it, int i) -> const float* {
    const int t = A.t0 + it;
    const int tn = trades(MODE) ? t + 1 : A.t0;
    if (i < D) return C.close + static_cast<size_t>(t) * D + i;
    if (i < 2 * D) return C.close + static_cast<size_t>(tn) * D + (i - D);
    if (i < n_mkt) return C.ind + static_cast<size_t>(tn) * C.I * D + (i - 2 * D);
    return A.act + (static_cast<size_t>(it) * N + n0) * D + (i - n_mkt);
  };
  constexpr int NSTAGE = OCC >= 4 ? kStage / 4 : OCC >= 3 ? kStage / 2 : kStage;
  float stage[NSTAGE];
  auto fetch_issue = [&](int it) {
#pragma unroll
    for (int j = 0; j < NSTAGE; ++j) {
      const int i = lane + kWave * j;
      stage[j] = (i < staged && (i >= D || trades(MODE))) ? *src_of(it, i) : 0.0f;
    }
  };
  auto fetch_commit = [&](int it) {
    float* buf = s_in0 + (it % kInBufs) * IB;
#pragma unroll
    for (int j = 0; j < NSTAGE; ++j) {
      const int i = lane + kWave * j;
      if (i < staged) buf[i] = stage[j];
    }
    for (int i = staged + lane; i < total; i += kWave) buf[i] = *src_of(it, i);  // large tiles
  };

  if (role == 2) {
    fetch_issue(0);
    fetch_commit(0);
    if (n_iter > 1) fetch_issue(1);
  }
  __syncthreads();

  for (int it = 0; it <= n_iter; ++it) {
    if (role == 0) {
      if (it < n_iter) {
        const int t = A.t0 + it;
        float* in = s_in0 + (it % kInBufs) * IB;
        CL.act = in + n_mkt;
        CL.px = in;
        CL.pn = in + D;
        CL.hold = s_hold;
        CL.qty = s_qty0 + (it & 1) * QB;
        CL.env = s_env0 + (it & 1) * EB;
        double* s_rew = s_rew0 + (it & 1) * RB;
        if (MODE == kEnsemble) {
          float* act = in + n_mkt;
          // Noise: one Philox block per (env, group of 4 stocks).
          const int G = (D + 3) >> 2;
          const float inv_g = 1.0f / static_cast<float>(G);
          const float inv_d = 1.0f / static_cast<float>(D);
          if (A.sigma != 0.0f) {
            for (int i = lane; i < M * G; i += kWave) {
              const int m = div_small(i, inv_g);
              const int g = i - m * G;
              float z[4];
              noise_block(A.noise_key, static_cast<uint64_t>(A.env_offset + n0 + m),
                          static_cast<uint64_t>(t), static_cast<uint64_t>(g), z);
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (4 * g + r < D) s_eps[m * D + 4 * g + r] = z[r];
            }
          }
          wave_lds_sync();
          for (int i = lane; i < MD; i += kWave) {
            float acc = 0.0f;
            for (int k = 0; k < A.K; ++k)
              acc = acc + A.mix[k] * A.mu[(static_cast<size_t>(k) * N + n0) * D + i];
            float a = acc;
            if (A.sigma != 0.0f) a = acc + A.sigma * s_eps[i];
            a = fminf(fmaxf(a, -1.0f), 1.0f);
            act[i] = a;
          }
          (void)inv_d;
        }
        // The chain: parallel pre-terms, serial cash recurrence per env, parallel post-terms.
        wave_lds_sync();
        if (trades(MODE)) {
          chain_day_terms(CL, Z, lane, kWave, C.one_p);
          chain_pairs_a(CL, Z, M, lane, kWave, C.hmax_f, C.one_m, C.one_p);
          wave_lds_sync();
          if (active)
            chain_serial<OCC == 1 ? 8 : 4, (OCC < 4)>(cash, CL.pro + lane * Z.RD, CL.deb + lane * Z.RD, CL.c1, CL.rc1, CL.qd + lane * Z.RI, CL.px,
                         CL.kq + lane * Z.RI, Z.DP, C.one_p);
          wave_lds_sync();
          chain_pairs_c(CL, Z, M, lane, kWave, C.hold_scale);
        } else {
          chain_pairs_hold(CL, Z, M, lane, kWave, C.hold_scale);
        }
        wave_lds_sync();
        if (active) {
          const double v_new = chain_value(cash, CL.val + lane * Z.RD, Z.DP);
          if (trades(MODE)) {
            const double r = (v_new - asset) * C.reward_scale;
            cumrew = cumrew + r;
            s_rew[lane] = r;
          }
          if (MODE != kObserve) asset = v_new;
          CL.env[lane * DS] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
        }
      }
    } else if (role == 1) {
      if (it >= 1) {
        // Results of step j = it - 1: the tile's rows are contiguous in every [N][.] trajectory.
        const int j = it - 1;
        const float* in = s_in0 + (j % kInBufs) * IB;
        const int* qty = s_qty0 + (j & 1) * QB;
        const float* env = s_env0 + (j & 1) * EB;
        const size_t row0 = static_cast<size_t>(j) * N + n0;
        if (trades(MODE)) {
          const double* s_rew = s_rew0 + (j & 1) * RB;
          if (A.rew && lane < M) A.rew[row0 + lane] = s_rew[lane];
          if (MODE == kEnsemble && A.act_out)
            wave_store_row(A.act_out + row0 * D, MD, lane, [&](int i) { return in[n_mkt + i]; });
          if (A.qty) wave_store_row(A.qty + row0 * D, MD, lane, [&](int i) { return qty[i]; });
        }
        if (A.obs) store_state_rows(A.obs + row0 * S, M, S, D, env, DS, in, C.price_scale, lane);
      }
    } else {
      if (it + 1 < n_iter) {
        fetch_commit(it + 1);
        if (it + 2 < n_iter) fetch_issue(it + 2);
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

template <int MODE, int OCC>
hipError_t launch_tile(const EnvConst& C, const EnvState& st, const StepArgs& A, size_t lds, int grid,
                       hipStream_t stream) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(env_tile_kernel<MODE, OCC>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((env_tile_kernel<MODE, OCC>), dim3(grid), dim3(3 * kWave), lds, stream, C, st, A);
  return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_tile(const EnvConst& C, const EnvState& st, StepArgs A, hipStream_t stream) {
  A.M = max(1, min(A.M, 64));
  while (A.M > 1 && tile_lds_bytes(A.M, C.D, C.I) > kMaxLds) A.M /= 2;
  const size_t lds = tile_lds_bytes(A.M, C.D, C.I);
  if (lds > kMaxLds) return hipErrorInvalidValue;
  const int grid = (C.N + A.M - 1) / A.M;
  // Two workgroups per compute unit when there are more tiles than compute units and two fit.
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 0;
  if (cus > 0 && grid > 3 * cus && 4 * lds <= kMaxLds) return launch_tile<MODE, 4>(C, st, A, lds, grid, stream);
  if (cus > 0 && grid > 2 * cus && 3 * lds <= kMaxLds) return launch_tile<MODE, 3>(C, st, A, lds, grid, stream);
  if (cus > 0 && grid > cus && 2 * lds <= kMaxLds) return launch_tile<MODE, 2>(C, st, A, lds, grid, stream);
  return launch_tile<MODE, 1>(C, st, A, lds, grid, stream);
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
